"""Sub-tile shapes of the tiled kernel and their autotuner.

Every shape gives the same X0 and X1 bit for bit: each output block sums its
products over the same common columns in the same order, whatever the
grouping of outputs into workgroups (only the order of the per-workgroup
trace partial sums changes).  The tuner records its choice in the cache file,
and a context that finds its key there takes the shape without timing."""
import json

import numpy as np
import pytest

from paper_2009_03551_amd import tc2 as T
from paper_2009_03551_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPE_ID = {"8x8": 0, "4x8": 1, "8x4": 2, "4x4": 3}
KIND_ID = {"fp64": 0, "fp32": 1, "bf16": 2, "fp32w": 3}


def default_shape(kind, D):
    # the default of a problem with at least as many cluster pairs as compute
    # units (smaller FP64 problems take 4x8; the cache below names every kind)
    return "4x4" if kind in ("fp64", "fp32w") and D >= 2 else "8x8"


def cache_file(tmp_path, kind, D, b, skip, shape):
    """A cache that forces `shape` on `kind` and the default shape on the other
    kinds (a closing pair runs the FP64 kind, a BF16 solve the FP32 one)."""
    path = tmp_path / f"tune_{kind}_{D}_{shape}.jsonl"
    lines = []
    for k in KIND_ID:
        key = f"gfx950/{k}/D{D}/k{(b + 3) // 4}/s{skip}"
        lines.append(json.dumps({"key": key, "shape": shape if k == kind else default_shape(k, D),
                                 "ms": {}}))
    path.write_text("\n".join(lines) + "\n")
    return str(path)


def system(D):
    return W.config_system("cube10", L=4) if D == 1 else W.config_system("cube20", L=3)


def variant(kind):
    return {"fp64": dict(precision="fp64"),
            "fp32": dict(precision="fp32", closing_fp64=2),
            "bf16": dict(precision="bf16", closing_fp64=2),
            "fp32w": dict(precision="fp32", closing_fp64=2, wide=True)}[kind]


def same_results(a, b):
    assert a.branches == b.branches and a.iters == b.iters
    for x, y in zip([a.X0] + a.X1, [b.X0] + b.X1):
        assert np.array_equal(x.row_ptr, y.row_ptr) and np.array_equal(x.col, y.col)
        assert np.array_equal(x.val, y.val)
    for x, y in zip(a.alpha, b.alpha):
        assert abs(x - y) <= 1e-12 * abs(y)


@pytest.mark.parametrize("kind,D,shape", [
    ("fp64", 1, "8x8"), ("fp64", 1, "4x8"), ("fp64", 1, "8x4"),
    ("fp32", 1, "4x8"), ("fp32", 1, "8x4"), ("fp32", 3, "4x8"),
    ("fp32w", 1, "4x8"), ("fp32w", 1, "8x4"),
    ("bf16", 1, "4x8"), ("bf16", 3, "4x8"),
])
def test_every_shape_gives_the_same_matrices(tmp_path, kind, D, shape):
    s = system(D)
    ref = T.solve(s, **variant(kind))[0]
    path = cache_file(tmp_path, kind, D, s.H.b, 0, shape)
    got = T.solve(s, tune=True, tune_cache=path, **variant(kind))[0]
    print(f"  {kind} D={D} {shape}: shapes used {got.tile_shape} it={got.iters}", flush=True)
    assert got.tile_shape[KIND_ID[kind]] == SHAPE_ID[shape]
    assert got.ms_tune == 0.0                     # taken from the cache, not timed
    same_results(got, ref)


def test_tuner_times_records_and_reuses(tmp_path):
    s = W.config_system("cube10", L=5)
    path = str(tmp_path / "tune.jsonl")
    ref = T.solve(s, skip="bound")[0]
    first = T.Solver(s, skip="bound", tune=True, tune_cache=path)
    a = first.run()[0]
    b = first.run()[0]                            # same context: no second timing
    first.close()
    lines = [json.loads(x) for x in open(path).read().splitlines()]
    print(f"  tuned: {lines} shapes {a.tile_shape} tune {a.ms_tune:.2f} ms", flush=True)
    assert a.ms_tune > 0.0 and b.ms_tune == 0.0
    assert len(lines) == 1 and lines[0]["key"] == f"gfx950/fp64/D1/k4/s1"
    assert SHAPE_ID[lines[0]["shape"]] == a.tile_shape[0]
    assert set(lines[0]["ms"]) == {"8x8", "4x8", "8x4"}
    same_results(a, ref)
    c = T.solve(s, skip="bound", tune=True, tune_cache=path)[0]
    assert c.ms_tune == 0.0 and c.tile_shape[0] == a.tile_shape[0]
    same_results(c, ref)
