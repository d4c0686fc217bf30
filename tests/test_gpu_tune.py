"""Tune tables: per-length entries, the text loader, the environment override.

Launch shapes never change the bits of the bit-exact operations; reductions
change only through the order of their compensated additions.
"""

import os

import numpy as np
import pytest
import torch

from oracle import ops

pytestmark = pytest.mark.gpu

import paper_2009_10917_amd as bs  # noqa: E402
from gpu_util import bits, dev_uniform, scalar_out, to_host  # noqa: E402

TABLE = """# test table
copy f64 0 1 1073741824 0
copy f64 4096 2 1024 0
copy f64 100000 8 64 0   # trailing comment
dot f64 0 4 256 0
"""


def test_entries_by_length(ctx, tmp_path):
    c = bs.bs_ctx_create(0)
    p = tmp_path / "t.txt"
    p.write_text(TABLE)
    assert bs.bs_ctx_load_tune(c, p) == 4
    assert bs.bs_ctx_tune_for(c, "copy", 0) == (1, 1 << 30, 0)
    assert bs.bs_ctx_tune_for(c, "copy", 4095) == (1, 1 << 30, 0)
    assert bs.bs_ctx_tune_for(c, "copy", 4096) == (2, 1024, 0)
    assert bs.bs_ctx_tune_for(c, "copy", 10 ** 9) == (8, 64, 0)
    assert bs.bs_ctx_tune_for(c, "dot", 10 ** 9) == (4, 256, 0)
    # other dtypes and operations keep their entries
    fresh = bs.bs_ctx_create(0)
    for n in (0, 10 ** 5, 10 ** 9):
        assert bs.bs_ctx_tune_for(c, "copy", n, dtype=bs.BS_F32) == bs.bs_ctx_tune_for(fresh, "copy", n, dtype=bs.BS_F32)
        assert bs.bs_ctx_tune_for(c, "norm", n) == bs.bs_ctx_tune_for(fresh, "norm", n)
    fresh.close()
    bs.bs_ctx_set_tune_entry(c, "copy", 50000, 4, 128)
    assert bs.bs_ctx_tune_for(c, "copy", 60000) == (4, 128, 0)
    assert bs.bs_ctx_tune_for(c, "copy", 200000) == (8, 64, 0)
    # copy across the buckets gives the same bits
    for n in (100, 5000, 70000, 300001):
        x = dev_uniform(n, 1)
        y = torch.zeros_like(x)
        bs.bs_copy(c, x, y)
        assert torch.equal(x.view(torch.int64), y.view(torch.int64))
    x, y = dev_uniform(300001, 1), dev_uniform(300001, 2)
    o = scalar_out()
    bs.bs_dot(c, x, y, o)
    S = ops.dot(to_host(x), to_host(y))
    assert abs(float(to_host(o)[0]) - S) <= 1e-14 * float(np.sum(np.abs(to_host(x) * to_host(y))))
    c.close()


@pytest.mark.parametrize("text", [
    "copy f64 0 1 1024\n",                 # missing field
    "copy f64 0 3 1024 0\n",               # unroll
    "copy f99 0 1 1024 0\n",               # dtype
    "paste f64 0 1 1024 0\n",              # operation
    "copy f64 16 1 1024 0\n",              # no n_min 0
    "gather f64 0 1 1024 3\n",             # variant
    "scatter f64 0 1 1024 12\n",           # both workgroup-order flags
    "copy f64 0 1 1024 0 extra\n",         # trailing text
])
def test_malformed_tables_change_nothing(ctx, tmp_path, text):
    c = bs.bs_ctx_create(0)
    before = bs.bs_ctx_tune_for(c, "copy", 10 ** 6)
    p = tmp_path / "bad.txt"
    p.write_text("dot f64 0 2 512 0\n" + text)
    with pytest.raises(bs.BSError):
        bs.bs_ctx_load_tune(c, p)
    assert bs.bs_ctx_tune_for(c, "copy", 10 ** 6) == before
    assert bs.bs_ctx_tune_for(c, "dot", 0) != (2, 512, 0)
    c.close()


def test_environment_override(tmp_path, monkeypatch):
    p = tmp_path / "env.txt"
    p.write_text("axpy f32 0 2 2048 0\n")
    monkeypatch.setenv("BS_TUNE_FILE", str(p))
    c = bs.bs_ctx_create(0)
    assert bs.bs_ctx_tune_for(c, "axpy", 10, dtype=bs.BS_F32) == (2, 2048, 0)
    c.close()
    monkeypatch.setenv("BS_TUNE_FILE", "none")
    c = bs.bs_ctx_create(0)
    assert bs.bs_ctx_tune_for(c, "axpy", 10, dtype=bs.BS_F32) == (1, 1 << 30, 0)
    c.close()
    monkeypatch.setenv("BS_TUNE_FILE", str(tmp_path / "missing.txt"))
    with pytest.raises(bs.BSError):
        bs.bs_ctx_create(0)


def test_installed_table_loads(ctx):
    path = os.path.join(os.path.dirname(bs.LIB_PATH), "tune_gfx950.txt")
    if not os.path.exists(path):
        pytest.skip("no tune table installed beside the library")
    c = bs.bs_ctx_create(0)
    assert bs.bs_ctx_load_tune(c, path) > 0
    c.close()


def test_reset_restores_the_table_set_tune_replaced():
    # bs_ctx_set_tune leaves one entry for every length; bs_ctx_reset_tune
    # brings back what bs_ctx_create set up, length by length
    fresh = bs.bs_ctx_create(0)
    c = bs.bs_ctx_create(0)
    lengths = (1, 1 << 16, 1 << 20, 1 << 24, 1 << 27, 1 << 30)
    ops = ("copy", "axpy", "norm", "dot", "cg_update", "gather", "scatter")
    want = {(op, d, n): bs.bs_ctx_tune_for(fresh, op, n, d) for op in ops for d in (0, 1, 2) for n in lengths}
    for op in ops:
        bs.bs_ctx_set_tune(c, op, 2, 1024, 1 if op in ("gather", "scatter") else 0)
    bs.bs_ctx_reset_tune(c)
    got = {(op, d, n): bs.bs_ctx_tune_for(c, op, n, d) for op in ops for d in (0, 1, 2) for n in lengths}
    assert got == want
    fresh.close()
    c.close()
