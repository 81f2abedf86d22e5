"""Continuous-batching request loop (run on an MI355X)."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_serving_overlap_and_alone_equals_mix(lib):
    from paper_2103_08473_amd import exacc
    from paper_2103_08473_amd.serve import Request, _make_inputs, report, run_stream, solve_one
    shapes = [(4, 24, 72, 11), (6, 36, 108, 12), (5, 40, 120, 13), (8, 48, 144, 14), (3, 21, 63, 15),
              (7, 42, 126, 16)]
    reqs = [Request(k, o, v, X, s) for k, (o, v, X, s) in enumerate(shapes)]
    opts = dict(precision=exacc.MIXED_FP32, tol=1e-8, max_iter=80)
    t_sum = sum(exacc.memory_estimate(o, v, X, precision=exacc.MIXED_FP32) for o, v, X, _ in shapes)
    budget = int(0.6 * t_sum)           # forces queueing on memory, not only on slots
    srv = run_stream(reqs, rate=50.0, hbm_budget=budget, max_active=4, opts=opts, producers=2)
    rep = report(srv.done, max(r.finished for r in srv.done))
    print(rep, flush=True)
    sys.stdout.flush()
    assert rep["converged"] == len(shapes), rep["failed"]
    # requests overlapped: some request was admitted before another finished
    done = sorted(srv.done, key=lambda r: r.admitted)
    assert any(b.admitted < a.finished for a, b in zip(done, done[1:]))
    # and memory admission made some wait
    assert any(r.admitted - r.arrival > 0.05 for r in srv.done)
    for r in srv.done:
        alone = Request(r.k, r.nocc, r.nvir, r.naux, r.seed)
        alone.inputs = _make_inputs((r.nocc, r.nvir, r.naux, r.seed))
        solve_one(alone, opts)
        assert alone.iterations == r.iterations
        assert alone.energy == r.energy      # deterministic kernels: bitwise identical


def test_request_over_budget_is_rejected_not_run(lib):
    from paper_2103_08473_amd import exacc
    from paper_2103_08473_amd.serve import Request, run_stream
    reqs = [Request(0, 4, 24, 72, 3)]
    srv = run_stream(reqs, rate=0, hbm_budget=1 << 20, max_active=2, opts=dict(precision=exacc.FP64),
                     producers=1)
    assert srv.done[0].status == exacc.ERR_NOMEM and not srv.done[0].converged
