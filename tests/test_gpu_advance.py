"""tc2_advance (a solve run in pieces), the per-update metrics log, row export
and the device-side comparison of iterates, through the C ABI.

A solve advanced in pieces runs the same kernels in the same order as
tc2_run, and every reduction is taken in a fixed order, so its results are
bitwise identical to a whole solve.  The exports and the comparison are
checked against the full host export of the same iterate.
"""
import json

import numpy as np
import pytest

from oracle import tc2_oracle as O
from paper_2009_03551_amd import tc2 as T
from paper_2009_03551_amd import workloads as W

pytestmark = pytest.mark.gpu

BENCH_VARIANT = dict(precision="fp32", wide=True, fp64_first=4, closing_fp64=2, skip="bound",
                     graph=True)


def same_result(a, b):
    assert a.status == b.status and a.iters == b.iters and a.branches == b.branches
    assert a.alpha == b.alpha and a.e0 == b.e0 and a.tr_x0 == b.tr_x0
    for x, y in zip([a.X0] + a.X1, [b.X0] + b.X1):
        assert np.array_equal(x.row_ptr, y.row_ptr) and np.array_equal(x.col, y.col)
        assert np.array_equal(x.val, y.val)


@pytest.mark.parametrize("name,kw,variant", [
    ("chain64", dict(n=24), dict(precision="fp64", graph=True)),
    ("cube10", dict(L=4, n_dir=3), BENCH_VARIANT),
])
def test_pieces_equal_a_whole_solve(name, kw, variant):
    s = W.config_system(name, **kw)
    whole = T.solve(s, **variant)[0]
    print(f"  {name}: {whole.status_name} {whole.iters} {whole.branches}", flush=True)
    sv = T.Solver(s, **variant)
    try:
        n = whole.iters
        assert n > 6
        for piece in (1, 2, 3):
            p, r = sv.advance(piece)
            assert p["updates"] == piece and r is None and p["solve_open"]
        # the last update of the solve finishes it within the same call
        p, r = sv.advance(n - 6)
        assert p["updates"] == n - 6 and p["solves_completed"] == 1 and not p["solve_open"]
        same_result(r[0], whole)
        # across a solve boundary: the next solve begins from H and repeats the first
        p, r = sv.advance(n + 3)
        assert p["updates"] == n + 3 and p["solves_completed"] == 1 and p["solve_open"]
        same_result(r[0], whole)
        p, r = sv.advance(n - 3)
        assert p["updates"] == n - 3 and p["solves_completed"] == 1 and not p["solve_open"]
        same_result(r[0], whole)
        # tc2_run after a partial advance starts again from H
        sv.advance(2)
        same_result(sv.run()[0], whole)
    finally:
        sv.close()


def test_metrics_log_has_every_update(tmp_path):
    s = W.config_system("chain64", n=24)
    path = str(tmp_path / "m.jsonl")
    g = T.solve(s, precision="fp64", metrics_log=path)[0]
    o = O.solve_system(s, keep_history=True)
    lines = [json.loads(x) for x in open(path)]
    assert [x["update"] for x in lines] == list(range(1, g.iters + 1))
    assert "".join(x["branch"] for x in lines) == g.branches == o.branches
    for x, h in zip(lines, o.history):
        assert x["tr_x0"] == pytest.approx(h["tr"], rel=1e-12)
        assert x["e0"] == pytest.approx(h["E0"], rel=1e-12)
        assert x["alpha"][0] == pytest.approx(h["alpha"][0], rel=1e-10)
        assert x["iota"] == pytest.approx(h["iota"], abs=1e-10)
        assert x["kind"] == "fp64" and x["system"] == 0 and x["solve"] == 1
    assert lines[-1]["active"] is False and lines[-1]["status"] == g.status
    assert all(x["active"] for x in lines[:-1])
    assert lines[-1]["nnzb"] == g.kept_blocks


def test_export_rows_equals_the_full_export():
    s = W.config_system("cube10", L=4, n_dir=2)
    sv = T.Solver(s, precision="fp32", wide=True, fp64_first=2, closing_fp64=2, export=True)
    try:
        g = sv.run()[0]
        rows = [5, 0, 63, 21]
        x0, x1 = sv.export_rows(0, rows)
        for got, full in zip([x0] + x1, [g.X0] + g.X1):
            for I in range(s.H.nb):
                a0, a1 = int(got.row_ptr[I]), int(got.row_ptr[I + 1])
                if I not in rows:
                    assert a1 == a0
                    continue
                f0, f1 = int(full.row_ptr[I]), int(full.row_ptr[I + 1])
                assert np.array_equal(got.col[a0:a1], full.col[f0:f1])
                assert np.array_equal(got.val[a0:a1], full.val[f0:f1])
    finally:
        sv.close()


def test_export_rows_of_a_batch_member():
    systems = W.batch_systems(n_sys=3, lo=30, hi=70, seed=9, n_dir=1)
    sv = T.Solver(systems, precision="fp64", export=True)
    try:
        g = sv.run()
        for k, sy in enumerate(systems):
            rows = [0, sy.H.nb - 1]
            x0, x1 = sv.export_rows(k, rows)
            for I in rows:
                a0, a1 = int(x0.row_ptr[I]), int(x0.row_ptr[I + 1])
                f0, f1 = int(g[k].X0.row_ptr[I]), int(g[k].X0.row_ptr[I + 1])
                assert np.array_equal(x0.col[a0:a1], g[k].X0.col[f0:f1])
                assert np.array_equal(x1[0].val[a0:a1], g[k].X1[0].val[f0:f1])
    finally:
        sv.close()


def merged_entries(results, m):
    """(rows, cols, vals) of matrix m of a batch's host results, merged."""
    rows, cols, vals, off = [], [], [], 0
    for r in results:
        X = r.X0 if m == 0 else r.X1[m - 1]
        rr = np.repeat(np.arange(X.nb), np.diff(X.row_ptr))
        rows.append(rr + off)
        cols.append(X.col + off)
        vals.append(X.val)
        off += X.nb
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def host_maxdiff(a, b):
    ka = a[0].astype(np.int64) * 10 ** 7 + a[1]
    kb = b[0].astype(np.int64) * 10 ** 7 + b[1]
    _, ia, ib = np.intersect1d(ka, kb, assume_unique=True, return_indices=True)
    d = np.abs(a[2][ia] - b[2][ib]).max() if len(ia) else 0.0
    oa = np.setdiff1d(np.arange(len(ka)), ia)
    ob = np.setdiff1d(np.arange(len(kb)), ib)
    if len(oa):
        d = max(d, np.abs(a[2][oa]).max())
    if len(ob):
        d = max(d, np.abs(b[2][ob]).max())
    return float(d)


def test_entries_export_and_device_compare():
    systems = W.batch_systems(n_sys=2, lo=40, hi=90, seed=11, n_dir=2)
    ref = T.Solver(systems, precision="fp64", export=True)
    var = T.Solver(systems, precision="fp32", closing_fp64=2, export=True)
    try:
        gr, gv = ref.run(), var.run()
        n = ref.iterate_size()
        assert n == sum(int(r.X0.row_ptr[-1]) for r in gr)
        for m in range(3):
            # export in two pieces, as the benchmark does in chunks
            a = ref.export_entries(m, 0, n // 3)
            b_ = ref.export_entries(m, n // 3, n - n // 3)
            rows = np.concatenate([a[0], b_[0]])
            cols = np.concatenate([a[1], b_[1]])
            vals = np.concatenate([a[2], b_[2]])
            want = merged_entries(gr, m)
            assert np.array_equal(rows, want[0]) and np.array_equal(cols, want[1])
            assert np.array_equal(vals, want[2])
            # the same iterate compares to zero; the other variant to the host diff
            assert ref.compare_entries(m, rows, cols, vals) == 0.0
            dv = var.compare_entries(m, rows, cols, vals)
            hv = host_maxdiff(want, merged_entries(gv, m))
            print(f"  matrix {m}: device {dv:.3e} host {hv:.3e}", flush=True)
            assert dv == hv and dv > 0.0
            # a missing entry on the caller's side counts as zero there
            keep = np.ones(len(rows), dtype=bool)
            keep[len(rows) // 2] = False
            dmiss = ref.compare_entries(m, rows[keep], cols[keep], vals[keep])
            assert dmiss == np.abs(vals[len(rows) // 2]).max()
    finally:
        ref.close()
        var.close()


def test_pool_kept_across_contexts_and_trimmed_on_request():
    # a second context reuses the chunks the first one gave back; trimming the
    # pool in between changes nothing in the results
    s = W.config_system("cube10", L=5, n_dir=3, eps=1e-5)
    a = T.solve(s, precision="fp64", skip="bound", graph=True)[0]
    b = T.solve(s, precision="fp64", skip="bound", graph=True)[0]
    T.trim_memory(0)
    c = T.solve(s, precision="fp64", skip="bound", graph=True)[0]
    same_result(a, b)
    same_result(a, c)
    with pytest.raises(T.TC2Error):
        T.trim_memory(4096)
