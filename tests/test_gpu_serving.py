"""Continuous-batching request loop (run on an MI355X)."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_serving_overlap_and_alone_equals_mix(lib):
    """Six requests of different sizes served with four slots under an HBM budget of 60% of
    their summed footprints (mixed FP32, FP64 refinement to 1e-8): all converge; each served
    energy equals the oracle's converged energy within 1e-7 Eh and the same request solved
    alone, bitwise; admission made some wait; and the mix finished in less wall time than the
    requests take one after another, so their work overlapped."""
    import time
    import oracle
    from paper_2103_08473_amd import exacc
    from paper_2103_08473_amd.serve import Request, _make_inputs, report, run_stream, solve_one
    shapes = [(4, 24, 72, 11), (6, 36, 108, 12), (5, 40, 120, 13), (8, 48, 144, 14), (3, 21, 63, 15),
              (7, 42, 126, 16)]
    reqs = [Request(k, o, v, X, s) for k, (o, v, X, s) in enumerate(shapes)]
    opts = dict(precision=exacc.MIXED_FP32, tol=1e-8, max_iter=80, timing=1)
    t_sum = sum(exacc.memory_estimate(o, v, X, precision=exacc.MIXED_FP32) for o, v, X, _ in shapes)
    budget = int(0.6 * t_sum)           # forces queueing on memory, not only on slots
    warm = Request(99, 3, 21, 63, 15)   # code objects loaded before anything is timed
    warm.inputs = _make_inputs((3, 21, 63, 15))
    solve_one(warm, opts)
    srv = run_stream(reqs, rate=1000.0, hbm_budget=budget, max_active=4, opts=opts, producers=2)
    first = min(r.arrival for r in srv.done)
    makespan = max(r.finished for r in srv.done) - first
    rep = report(srv.done, makespan)
    print(rep, flush=True)
    sys.stdout.flush()
    assert rep["converged"] == len(shapes), rep["failed"]
    # requests overlapped: some request was admitted before another finished
    done = sorted(srv.done, key=lambda r: r.admitted)
    assert any(b.admitted < a.finished for a, b in zip(done, done[1:]))
    # and memory admission made some wait: a request at the head of the queue found a slot
    # free but not enough of the HBM budget
    assert any(r.mem_wait and r.admitted > r.arrival for r in srv.done)
    alone_wall = 0.0
    for r in sorted(srv.done, key=lambda r: r.k):
        eps, B = _make_inputs((r.nocc, r.nvir, r.naux, r.seed))
        alone = Request(r.k, r.nocc, r.nvir, r.naux, r.seed)
        alone.inputs = (eps, B)
        t0 = time.perf_counter()
        solve_one(alone, opts)
        alone_wall += time.perf_counter() - t0
        assert alone.iterations == r.iterations
        assert alone.energy == r.energy      # deterministic kernels: bitwise identical
        ref = oracle.solve(eps, B, r.nocc, max_iter=80, tol=1e-10)
        print("request %d (%d, %d, %d): |E - E_oracle| %.2e Eh, device %.0f ms" % (
            r.k, r.nocc, r.nvir, r.naux, abs(r.energy - ref.energy), r.device_ms), flush=True)
        assert ref.converged and abs(r.energy - ref.energy) <= 1e-7
    print("makespan %.2f s, requests one after another %.2f s" % (makespan, alone_wall), flush=True)
    assert makespan < alone_wall


def test_request_over_budget_is_rejected_not_run(lib):
    from paper_2103_08473_amd import exacc
    from paper_2103_08473_amd.serve import Request, run_stream
    reqs = [Request(0, 4, 24, 72, 3)]
    srv = run_stream(reqs, rate=0, hbm_budget=1 << 20, max_active=2, opts=dict(precision=exacc.FP64),
                     producers=1)
    assert srv.done[0].status == exacc.ERR_NOMEM and not srv.done[0].converged
