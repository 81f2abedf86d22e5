"""The C-ABI library loads and exports every symbol include/exacc.h declares (no GPU calls)."""
import ctypes

from paper_2103_08473_amd import exacc


def test_library_exports_every_declared_symbol():
    L = exacc.load()
    names = exacc.declared_symbols()
    assert "exacc_ccsd_create" in names and "exacc_ccsd_iterate" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_entry_points():
    """Functions that never touch the device: options, memory plan, flop count, status text."""
    o = exacc.default_opts()
    assert o.diis_size == 8 and o.max_iter == 30 and abs(o.tol - 1e-9) < 1e-24
    assert o.precision == exacc.FP64 and o.level_shift == 0.0
    m1 = exacc.memory_estimate(10, 40, 120)
    m2 = exacc.memory_estimate(40, 360, 1200)
    assert 0 < m1 < m2
    assert exacc.memory_estimate(0, 40, 120) == 0
    # ladder flops: 8 * (X sum_{m<=v} m^2 (m-1) + Po Pv^2): the Hermitian build (blocks on and
    # above the pair diagonal) by direct summation, plus the contraction
    Po, Pv = 40 * 39 / 2, 360 * 359 / 2
    build = 1200 * sum(m * m * (m - 1) for m in range(1, 361))
    assert abs(exacc.ladder_flops(40, 360, 1200) - 8 * (build + Po * Pv ** 2)) < 1e3
    # about half of the full build 2 X Pv^2
    assert abs(build / (2 * 1200 * Pv ** 2) - 0.5) < 0.01
    L = exacc.load()
    assert L.exacc_status_string(0) == b"ok"
    assert L.exacc_status_string(-2).startswith(b"out of device memory")
    assert L.exacc_ccsd_destroy(None) == 0


def test_create_rejects_bad_sizes_before_touching_the_device():
    L = exacc.load()
    h = ctypes.c_void_p()
    o = exacc.default_opts()
    assert L.exacc_ccsd_create(ctypes.byref(h), 0, 10, 10, None, None, ctypes.byref(o)) == -1
    assert not h.value
    assert b"nocc" in L.exacc_last_error()


def test_df_factors_rejects_bad_sizes_before_touching_the_device():
    L = exacc.load()
    it = ctypes.c_int(0)
    buf = (ctypes.c_double * 64)()
    # nspinor > nao, naux < 1, null pointers: refused by the host checks
    assert L.exacc_df_factors(3, 5, 2, buf, buf, buf, buf, 0, None, ctypes.byref(it)) == -1
    assert L.exacc_df_factors(3, 2, 0, buf, buf, buf, buf, 0, None, ctypes.byref(it)) == -1
    assert L.exacc_df_factors(3, 2, 2, None, buf, buf, buf, 0, None, ctypes.byref(it)) == -1
    assert b"DF factors" in L.exacc_last_error()


def test_new_options_default_to_automatic():
    o = exacc.default_opts()
    assert o.triples_occ_block == 0 and o.doubles_only == 0 and o.cc2 == 0
    assert o.ladder_defect_correction == 1 and o.graph_residual == 0 and o.ladder_group_nvir == 64


def test_grouped_ladder_scratch_is_planned():
    """With all ladder rows in one product (nvir <= ladder_group_nvir) the tile scratch holds
    v^4 complex elements instead of one row's v (v - 1) v; nothing else in the plan changes."""
    v = 40
    grouped = exacc.memory_estimate(6, v, 120)
    per_row = exacc.memory_estimate(6, v, 120, ladder_group_nvir=0)
    assert grouped - per_row == (v ** 4 - v * (v - 1) * v) * 16
    # above the threshold, or with a ladder chunk smaller than the pair range, per row
    assert exacc.memory_estimate(6, 65, 120) == exacc.memory_estimate(6, 65, 120, ladder_group_nvir=0)
    assert exacc.memory_estimate(6, v, 120, ladder_chunk_pairs=100) == \
        exacc.memory_estimate(6, v, 120, ladder_chunk_pairs=100, ladder_group_nvir=0)


def test_bench_runs_on_one_gpu_only():
    """bench.py --gpus N with N > 1 exits with a message (before any device work)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
