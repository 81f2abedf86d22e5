"""Benchmark: the CCSD amplitude iteration on one MI355X, FP64 and mixed precision.

A step is one pass of the whole iteration (eq. CC_general residual with the
particle ladder built from density-fitting tiles, ring, intermediates,
denominator step, DIIS, energy) for the nocc=40, nvir=360, naux=1200 system in
complex FP64, with the inputs resident in HBM before the timed region.  The
timed steps are iterations of a solve that then runs on to convergence.

Prints one JSON line:
  value         ladder algorithmic TFLOP per iteration (Hermitian tile build plus
                contraction, exacc_ladder_flops) / wall time of a whole FP64 iteration;
  roofline      the ladder tile-build kernel (the dominant kernel), timed with HIP
                events on the library's stream during the timed steps;
  solves        time to solution at ||Delta|| <= 1e-9 of the FP64, mixed FP32 and mixed
                BF16x3 schedules, their iterations (low precision + FP64), |dE| and
                max |dT| against the FP64 solve;
  serving       a Poisson stream of requests of the serving configuration (continuous
                batching, HBM admission), p50/p99 latency and solves/s;
  clock         the GPU shader clock sampled during each leg;
  cpu_baseline  the CPU oracle's particle-ladder term on a bounded sample of rows.
"""
from __future__ import annotations

import argparse
import glob
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA = 78.6  # TFLOP/s, MI355X dense FP64 matrix
PEAK_FP32_MFMA = 157.3  # TFLOP/s, MI355X dense FP32 matrix
PEAK_BF16_MFMA = 2516.6  # TFLOP/s, MI355X dense BF16 matrix
WORKLOAD = dict(nocc=40, nvir=360, naux=1200, seed=0)


# HBM bytes per ladder-build launch (mean over the launches of one iteration), from one
# rocprofv3 pass each of FETCH_SIZE and WRITE_SIZE, scaled by what the counters read for
# a plain 1 GiB device copy (fetch x2.000, write x1.000), and the kernel's MFMA-busy
# fraction and clock from a third pass.  They hold for the sources they were taken with:
# `source_sha256` hashes the FP64 part of gett.hip (up to the BF16x3 section) and the
# Hermitian ladder driver in exacc.cpp; the figures are reported as null once either
# text differs.
TRAFFIC = {"source_sha256": "92d536ddafb423d9bc33633bce1fb9315fdabc8b68f499c7b85fb7e9431cb068",
           "fetch_bytes": 4.5734e9, "write_bytes": 0.2123e9,
           "mfma_busy": 0.703, "clock_ghz": 2.34}
GETT_SRC = os.path.join(ROOT, "paper_2103_08473_amd", "csrc", "gett.hip")
EXACC_SRC = os.path.join(ROOT, "paper_2103_08473_amd", "csrc", "exacc.cpp")
BF16_MARK = b"// BF16x3 complex GETT"
LADDER_MARKS = (b"static void ladder_apply_herm(Handle& h, const Work<R>& w, const R* F, int64_t row_stride,\n"
                b"                              const TV<R>& Lp, R* Znp, bool bf, bool use_bvs) {",
                b"// The ring term of the FP64 iterations after a mixed-precision switch")


def kernel_source_sha256():
    import hashlib
    with open(GETT_SRC, "rb") as f:
        g = f.read()
    cut = g.find(BF16_MARK)
    with open(EXACC_SRC, "rb") as f:
        e = f.read()
    i, j = e.find(LADDER_MARKS[0]), e.find(LADDER_MARKS[1])
    return hashlib.sha256((g[:cut] if cut >= 0 else g) + (e[i:j] if 0 <= i < j else e)).hexdigest()


def measured_counters():
    """Counter-derived HBM bytes per launch and MFMA-busy figures, or None if the kernel or
    the ladder driver changed since they were taken."""
    if TRAFFIC["source_sha256"] is None or kernel_source_sha256() != TRAFFIC["source_sha256"]:
        return None
    return TRAFFIC


def ladder_build_flops(o, v, X):
    """Algorithmic flops of the Hermitian tile build: for each virtual a, (ac|bd) over
    c, d >= a, b > a (naux sum_m m^2 (m - 1), m = v - a), 8 per complex multiply-add."""
    return 8.0 * X * sum(m * m * (m - 1) for m in range(1, v + 1))


def ladder_build_bytes(o, v, X):
    """Mean algorithmic HBM bytes of one tile-build launch (FP64 complex) over the rows a:
    read the factor rows (a, c >= a) and (b > a, d >= a), write the (v-a) (v-a-1) (v-a) tile."""
    tot = 0.0
    for a in range(v - 1):
        m = v - a
        tot += 16.0 * (m * X + (m - 1) * m * X + m * (m - 1) * m)
    return tot / (v - 1)


class ClockSampler:
    """Samples the GPU's current shader clock (the active level of pp_dpm_sclk in sysfs)
    every 0.2 s on a host thread; legs are marked by name."""

    def __init__(self):
        self.path = None
        try:
            import torch
            p = torch.cuda.get_device_properties(0)
            bus = "%04x:%02x:%02x" % (getattr(p, "pci_domain_id", 0), p.pci_bus_id, p.pci_device_id)
            for f in glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk"):
                if bus in os.path.realpath(os.path.dirname(f)):
                    self.path = f
                    break
        except Exception:
            self.path = None
        self.samples, self.marks = [], []
        self.stop = threading.Event()
        self.t0 = time.perf_counter()
        if self.path:
            threading.Thread(target=self._run, daemon=True).start()

    def _read(self):
        with open(self.path) as f:
            for line in f:
                if line.rstrip().endswith("*"):
                    return float(line.split(":")[1].strip().split("Mhz")[0].split("MHz")[0])
        return None

    def _run(self):
        while not self.stop.is_set():
            try:
                mhz = self._read()
                if mhz is not None:
                    self.samples.append((time.perf_counter() - self.t0, mhz))
            except Exception:
                return
            self.stop.wait(0.2)

    def mark(self, name):
        self.marks.append((name, time.perf_counter() - self.t0))

    def report(self):
        import numpy as np
        self.stop.set()
        if not self.path:
            return {"source": None}
        out = {"source": self.path, "unit": "MHz"}
        ends = [t for _, t in self.marks[1:]] + [time.perf_counter() - self.t0]
        for (name, t0), t1 in zip(self.marks, ends):
            v = [m for t, m in self.samples if t0 <= t < t1]
            if v:
                out[name] = {"median": float(np.median(v)), "min": float(np.min(v)), "n": len(v)}
        return out


def host_info():
    import platform
    info = {"cpu_model": platform.processor() or "", "logical_cpus": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except Exception:
        pass
    try:
        import psutil
        info["physical_cores"] = psutil.cpu_count(logical=False)
    except Exception:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if blas:
            info["blas"] = "%s %s (%s), %d threads" % (blas[0].get("internal_api"), blas[0].get("version"),
                                                      blas[0].get("architecture"), blas[0].get("num_threads"))
            info["blas_threads"] = blas[0].get("num_threads")
    except Exception:
        pass
    return info


def cpu_baseline(eps, B, o, budget_s=15.0):
    """Time the oracle's particle-ladder rows on the host, until ~budget_s of work."""
    import numpy as np
    from oracle.ccsd import ladder_rows
    hi = host_info()
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
        m = v - rows
        # the same algorithmic work the GPU ladder counts for these rows: the Hermitian
        # tile build of row a plus its share of the contraction
        flops += 8.0 * (X * m * m * (m - 1) + Po * (m - 1) * Pv)
        rows += 1
    dt = time.perf_counter() - t0
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s",
            "cores": int(hi.get("blas_threads") or hi.get("affinity_cpus") or 1), "kind": "oracle",
            "host": hi,
            "sample": "oracle particle ladder (1/2 sum <ab||cd> tau_ij^cd, <ab||cd> built from B, "
                      "numpy complex128) for virtual rows a=0..%d of the 40/360/1200 system, %.1f s; "
                      "flops counted as the GPU ladder's algorithmic work for those rows" % (rows - 1, dt)}


def oracle_iteration(eps, B, o, ladder_rows_sample=6):
    """One-off timing of one oracle CCSD iteration on the host (CPU only).

    Timed whole: the oracle's integral classes (build_integrals) and its residual with the
    particle-ladder term set to zero (everything else of eq. CC_general), then the Jacobi
    step.  The ladder term, which does not fit in one run at this size, is timed on
    `ladder_rows_sample` of its rows a (each row builds <ab||cd> for all b, c, d and
    contracts it with tau: the same work for every a) and scaled to all v rows."""
    import types

    import numpy as np
    import oracle.ccsd as occ
    import oracle.integrals as oint
    hi = host_info()
    v = eps.size - o
    out = {"host": hi, "workload": "nocc=%d nvir=%d naux=%d" % (o, v, B.shape[0])}

    def say(msg):
        print("oracle iteration: " + msg, file=sys.stderr, flush=True)

    # the oracle's own einsum calls report each one that takes over 2 s as it ends (one
    # call of the residual takes minutes at this size)
    def einsum(spec, *ops, **kw):
        t = time.perf_counter()
        r = np.einsum(spec, *ops, **kw)
        dt = time.perf_counter() - t
        if dt > 2.0:
            say("einsum %s %.1f s" % (spec, dt))
        return r
    shim = types.SimpleNamespace(**{k: getattr(np, k) for k in dir(np) if not k.startswith("__")})
    shim.einsum = einsum
    saved = (occ.np, oint.np)
    occ.np, oint.np = shim, shim

    t0 = time.perf_counter()
    ints = occ.build_integrals(B, o)
    out["integrals_s"] = round(time.perf_counter() - t0, 2)
    say("integrals %.1f s" % out["integrals_s"])
    rng = np.random.default_rng(3)
    t1 = 1e-3 * (rng.standard_normal((o, v)) + 1j * rng.standard_normal((o, v)))
    t2 = 1e-3 * (rng.standard_normal((o, o, v, v)) + 1j * rng.standard_normal((o, o, v, v)))
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    full_ladder = occ._ladder
    occ._ladder = lambda ints_, tau_: np.zeros(tau_.shape, dtype=np.complex128)
    try:
        t0 = time.perf_counter()
        S1, S2 = occ.residual(eps, ints, t1, t2)
        d1, d2 = occ.denominators(eps, o)
        occ.jacobi_step(S1, S2, d1, d2)
        out["residual_without_ladder_s"] = round(time.perf_counter() - t0, 2)
    finally:
        occ._ladder = full_ladder
    say("residual without the ladder %.1f s" % out["residual_without_ladder_s"])
    del S1, S2
    tau = occ.tau(t1, t2)
    rows = np.linspace(0, v - 1, ladder_rows_sample).astype(int)
    t0 = time.perf_counter()
    for a in rows:
        occ.ladder_rows(ints["B"], o, tau, int(a), int(a) + 1)
        say("ladder row %d done" % a)
    per_row = (time.perf_counter() - t0) / len(rows)
    out["ladder_rows_timed"] = [int(a) for a in rows]
    out["ladder_s_per_row"] = round(per_row, 3)
    out["ladder_s"] = round(per_row * v, 1)
    say("ladder %.2f s per row, %.0f s for %d rows" % (per_row, per_row * v, v))
    out["iteration_s"] = round(out["residual_without_ladder_s"] + out["ladder_s"], 1)
    occ.np, oint.np = saved
    return out


def solve_leg(exacc, eps_d, B_d, o, stream, precision, tol, max_iter, progress, steps=0, warmup=0,
              stop_after_timed=False):
    """One solve to convergence from create; optionally the `steps` iterations after
    `warmup` are the timed FP64 steps (stop_after_timed: end there, for profiler runs).
    Returns a dict and the handle (open)."""
    import torch
    t_start = time.perf_counter()
    cc = exacc.CCSD(eps_d, B_d, o, stream=stream.cuda_stream, timing=1, tol=tol, max_iter=max_iter,
                    precision=precision)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t_start
    hist, phases = [], []
    timed = None
    low_stages = None  # stage times of the low-precision phase (mixed schedules)
    conv = False
    cc.stage_times(reset=True)
    while len(hist) < max_iter and not conv:
        k = len(hist)
        if steps and k == warmup:  # the timed steps: bracketed by device synchronisation
            cc.stage_times(reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                st, n, r, conv = cc.iterate(1)
                hist.append((len(hist) + 1, cc.energy(), r))
            torch.cuda.synchronize()
            timed = (time.perf_counter() - t0, cc.stage_times(reset=True), r)
            if stop_after_timed:
                break
            continue
        state = cc.phase()[0]  # 1 low precision, 2 corrected ladder, 0 FP64
        ti = time.perf_counter()
        st, n, r, conv = cc.iterate(1)
        phases.append((state, time.perf_counter() - ti))
        hist.append((len(hist) + 1, cc.energy(), r))
        if state == 1 and cc.phase()[0] != 1:
            low_stages = cc.stage_times(reset=True)
        if st == exacc.ERR_DIVERGED:
            break
    torch.cuda.synchronize()
    tts = time.perf_counter() - t_start
    e = cc.energy()
    _, n64 = cc.phase()
    progress("  %d iterations, %.1f s, converged %s" % (len(hist), tts, conv))
    def per(state):
        t = [dt for st_, dt in phases if st_ == state]
        return len(t), (round(sum(t) / len(t), 4) if t else None)
    n_low, s_low = per(1)
    n_dc, s_dc = per(2)
    return {"converged": bool(conv), "iterations": len(hist), "low_precision_iterations": n_low,
            "s_per_low_iter": s_low, "corrected_ladder_iterations": n_dc, "s_per_corrected_iter": s_dc,
            "final_fp64_iterations": int(n64), "time_to_solution_s": round(tts, 3),
            "create_s": round(t_create, 3), "energy": [e.real, e.imag],
            "residual_last": hist[-1][2] if hist else None,
            "low_stages": low_stages}, cc, timed


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="FP64 leg only")
    ap.add_argument("--no-solve", action="store_true",
                    help="FP64 timed steps only (no solve to convergence, no other leg): for profiler runs")
    ap.add_argument("--serving-requests", type=int, default=32)
    ap.add_argument("--serving-rate", type=float, default=0.29,
                    help="Poisson arrivals per second (0.8 x the 0.36 solves/s requests 0-127 of the "
                         "serving stream completed while the server was saturated)")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="first run one plain device-to-device copy of this many GiB (a known-size "
                         "kernel to scale hardware byte counters by)")
    ap.add_argument("--oracle-iteration", action="store_true",
                    help="only time one iteration of the CPU oracle at the benchmark size (no GPU; "
                         "about 10 minutes and 150 GB of host memory) and print it as JSON")
    args = ap.parse_args()
    if args.oracle_iteration:
        from paper_2103_08473_amd.synth import make_system
        o = WORKLOAD["nocc"]
        eps, B = make_system(o, WORKLOAD["nvir"], WORKLOAD["naux"], seed=WORKLOAD["seed"])
        print(json.dumps(oracle_iteration(eps, B, o)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2103_08473_amd import exacc
    from paper_2103_08473_amd.synth import make_system

    def progress(msg):
        print("bench: " + msg, file=sys.stderr, flush=True)

    o, v, X = WORKLOAD["nocc"], WORKLOAD["nvir"], WORKLOAD["naux"]
    progress("inputs")
    eps, B = make_system(o, v, X, seed=WORKLOAD["seed"])
    torch.cuda.set_device(0)
    clock = ClockSampler()
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
    tol = 1e-9

    # FP64 solve; its iterations warmup+1 .. warmup+steps are the timed steps
    progress("fp64 solve (timed steps %d after %d warm-up iterations)" % (args.steps, args.warmup))
    clock.mark("fp64")
    max_iter = max(80, args.warmup + args.steps)
    if args.no_solve:
        args.no_mixed = True
    s64, cc, timed = solve_leg(exacc, eps_d, B_d, o, stream, exacc.FP64, tol, max_iter, progress,
                               steps=args.steps, warmup=args.warmup, stop_after_timed=args.no_solve)
    dt, stages, res = timed
    s64.pop("low_stages", None)
    E = cc.energy()
    t1_64, t2_64 = cc.amplitudes() if not args.no_mixed else (None, None)

    extra = {}
    if not args.no_mixed:
        # Lambda equations (App. D) at the converged amplitudes: the first step also builds
        # the transformed-Hamiltonian pieces, so it is the warm-up
        progress("lambda iterations")
        clock.mark("lambda")
        cc.lambda_iterate(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nl = 3
        for _ in range(nl):
            cc.lambda_iterate(1)
        torch.cuda.synchronize()
        dtl = (time.perf_counter() - t0) / nl
        extra["lambda_fp64"] = {"s_per_iter": round(dtl, 4),
                                "ccsd_iteration_time_ratio": round((dt / args.steps) / dtl, 3)}
    cc.close()

    if not args.no_mixed:
        # CCD (the paper's CCDOUBLES) and CC2 variants: same system, FP64, 3 timed iterations
        for name, kw in (("ccd_fp64", {"doubles_only": 1}), ("cc2_fp64", {"cc2": 1})):
            progress(name)
            clock.mark(name)
            cd = exacc.CCSD(eps_d, B_d, o, stream=stream.cuda_stream, tol=tol, **kw)
            cd.iterate(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                cd.iterate(1)
            torch.cuda.synchronize()
            dtc = (time.perf_counter() - t0) / 3
            cd.close()
            extra[name] = {"s_per_iter": round(dtc, 4),
                           "ccsd_iteration_time_ratio": round((dt / args.steps) / dtc, 3)}

    solves = {"fp64": s64}
    if not args.no_mixed:
        for name, prec in (("mixed_fp32", exacc.MIXED_FP32), ("mixed_bf16x3", exacc.MIXED_BF16X3)):
            progress(name + " solve")
            clock.mark(name)
            sm, cm, _ = solve_leg(exacc, eps_d, B_d, o, stream, prec, tol, 80, progress)
            st = sm.pop("low_stages") or {}
            t1, t2 = cm.amplitudes()
            cm.close()
            e = complex(*sm["energy"])
            sm["abs_dE_vs_fp64_Eh"] = abs(e - E)
            sm["max_abs_dT1_vs_fp64"] = float(np.abs(t1 - t1_64).max())
            sm["max_abs_dT2_vs_fp64"] = float(np.abs(t2 - t2_64).max())
            sm["speedup_time_to_solution"] = round(s64["time_to_solution_s"] / sm["time_to_solution_s"], 3)
            nlow = max(1, sm["low_precision_iterations"])
            bms = st.get("ladder_build", float("nan"))
            sm["low_phase_ms_per_iter"] = {k: round(t / nlow, 2) for k, t in st.items()}
            if bms == bms:
                btf = ladder_build_flops(o, v, X) / (bms / nlow * 1e-3) / 1e12
                sm["low_phase_ladder_build_tflops"] = round(btf, 3)
                if prec == exacc.MIXED_FP32:
                    sm["low_phase_ladder_build_frac_fp32_peak"] = round(btf / PEAK_FP32_MFMA, 4)
                else:  # 12 bf16 MFMA products (24 flops) per complex multiply-add
                    sm["low_phase_ladder_build_hw_frac_bf16_peak"] = round(btf * 24 / 8 / PEAK_BF16_MFMA, 4)
            solves[name] = sm
            del t1, t2
        del t1_64, t2_64

        # DF-factor generation (the step before the iteration) for the same spinor count:
        # nao = 600 AO functions, nspinor = o + v = 400, naux = X.  Inputs made on the device
        # with torch (J = L K, V = L L^T, orthonormal C); not part of the timed product.
        try:
            progress("df factors")
            clock.mark("df_factors")
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
            extra["df_factors"] = {"nao": nao, "nspinor": nsp, "naux": X, "seconds": round(dtd, 4),
                                   "newton_schulz_steps": nsit, "tflops": round(fl / dtd / 1e12, 3),
                                   "flops_counted": "complex GEMM work, 8 flops per multiply-add"}
            del J, Vm, Cq, Bdf, Lm
            torch.cuda.empty_cache()
        except Exception as ex:  # the headline line must still print
            extra["df_factors"] = {"error": str(ex)[:200]}
    del B_d

    serving = None
    if not args.no_mixed and args.serving_requests > 0:
        from paper_2103_08473_amd.serve import Request, report, run_stream
        from paper_2103_08473_amd.synth import serving_request
        progress("serving stream of %d requests at %.3f/s" % (args.serving_requests, args.serving_rate))
        clock.mark("serving")
        reqs = [Request(k, *serving_request(k)) for k in range(args.serving_requests)]
        opts = dict(precision=exacc.MIXED_BF16X3, tol=1e-8, max_iter=80, timing=1)
        t0 = time.perf_counter()
        srv = run_stream(reqs, args.serving_rate, 200 << 30, 8, opts, producers=4)
        makespan = time.perf_counter() - t0
        serving = report(srv.done, makespan)
        busy = sum(r.device_ms for r in srv.done) * 1e-3
        serving.update({
            "config": "requests 0..%d of the serving stream: nocc ~ U{6..40}, nvir = round(r nocc), "
                      "r ~ U[5, 9], naux = 3 nvir, seed 1000+k; Poisson arrivals" % (args.serving_requests - 1),
            "rate_per_s": args.serving_rate, "precision": "mixed bf16x3, fp64 refinement to 1e-8",
            "max_active": 8, "hbm_budget_gb": 200,
            "stage_time_sum_over_makespan": round(busy / makespan, 3),
            "shapes": [[r.nocc, r.nvir, r.naux] for r in sorted(srv.done, key=lambda r: r.k)]})

    s_per_iter = dt / args.steps
    lad = exacc.ladder_flops(o, v, X)
    value = lad / s_per_iter / 1e12
    build_ms = stages.get("ladder_build", float("nan")) / args.steps
    contract_ms = stages.get("ladder_contract", float("nan")) / args.steps
    achieved = ladder_build_flops(o, v, X) / (build_ms * 1e-3) / 1e12
    ladder_ms = build_ms + contract_ms + stages.get("ladder_antisym", 0.0) / args.steps
    ctr = measured_counters()
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
        "residual_last_timed": res,
        "energy": [E.real, E.imag],
        "stage_ms_per_iter": {k: round(t / args.steps, 2) for k, t in stages.items()},
        "roofline": {"bound": "mfma", "kernel": "ladder tile build (GETT kind 1)",
                     "achieved": round(achieved, 3), "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_MFMA, 4),
                     "traffic": (ctr["fetch_bytes"] + ctr["write_bytes"]) if ctr else None,
                     "traffic_unit": "bytes per launch (HBM, counter-derived)",
                     "algorithmic_bytes_per_launch": round(ladder_build_bytes(o, v, X)),
                     "flops_counted": "8 real flops per complex multiply-add of the Hermitian build "
                                      "(blocks on and above the pair diagonal); the kernel's "
                                      "3-multiplication complex product issues 6",
                     "hw_frac": round(0.75 * achieved / PEAK_FP64_MFMA, 4),
                     "counters": ({"mfma_busy": ctr["mfma_busy"], "clock_ghz": ctr["clock_ghz"]}
                                  if ctr else None)},
        "solves": solves,
    }
    out.update(extra)
    if serving is not None:
        out["serving"] = serving
    out["clock"] = clock.report()
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(eps, B, o)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
