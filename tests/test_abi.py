"""The C ABI without a GPU: symbols, prototypes, host-side checks, host map."""

import ctypes
import os
import re

import numpy as np
import pytest

import bsgen
from oracle import mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bs.h")
LIB = os.path.join(ROOT, "paper_2009_10917_amd", "libbs.so")


def _ensure_built():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__._builder().build()


_ensure_built()
import paper_2009_10917_amd as bs  # noqa: E402


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    decls = re.findall(r"^\s*(?:const\s+)?\w+\*?\s+(bs_\w+)\s*\(([^;]*?)\)\s*;", text, flags=re.M | re.S)
    out = {}
    for name, args in decls:
        args = args.strip()
        out[name] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_every_declared_symbol_is_exported_with_matching_arity():
    decls = header_functions()
    assert len(decls) >= 20
    lib = ctypes.CDLL(LIB)
    for name, nargs in decls.items():
        assert hasattr(lib, name), name
        assert name in bs.PROTOTYPES, name
        assert len(bs.PROTOTYPES[name][1]) == nargs, name
    assert set(bs.PROTOTYPES) == set(decls)


def test_status_strings_and_version():
    for code, name in bs.STATUS_NAMES.items():
        assert bs.lib.bs_status_string(code).decode() == name
    assert "gfx950" in bs.bs_version()


def test_host_checks_reject_bad_arguments_before_any_launch():
    L = bs.lib
    INVALID = 1
    # NULL context: rejected on the host, nothing touches a device
    assert L.bs_copy(None, 0, 10, 16, 32, None) == INVALID
    assert b"ctx is NULL" in L.bs_last_error()
    assert L.bs_axpy(None, 0, 10, 1.0, 16, 1.0, 32, None) == INVALID
    assert L.bs_norm(None, 0, 10, 16, None, 64, None) == INVALID
    assert L.bs_dot(None, 0, 10, 16, 32, 64, None) == INVALID
    assert L.bs_cg_update(None, 0, 10, 1.0, 16, 32, 48, 64, None, 80, None) == INVALID
    assert L.bs_gather(None, None, 0, 16, 32, None) == INVALID
    assert L.bs_scatter(None, 0, 16, 16, 16, 32, 64, None) == INVALID
    assert L.bs_gs_scatter(None, None, 0, 16, 32, None) == INVALID
    assert L.bs_axpy_dev(None, 0, 10, 1.0, 16, None, 32, 1.0, None, None, 48, None) == INVALID
    assert L.bs_cg_update_dev(None, 0, 10, 1.0, 16, 24, 32, 48, 64, 80, None, 96, None) == INVALID
    # the context-free CG update validates before it looks up its buffer
    assert L.bs_cg_update_noalloc(0, 10, 1.0, None, 32, 48, 64, None, 80, None) == INVALID
    assert L.bs_cg_update_noalloc(7, 10, 1.0, 16, 32, 48, 64, None, 80, None) == INVALID
    assert L.bs_cg_update_noalloc(0, 10, 1.0, 16, 32, 48, 64, None, None, None) == INVALID
    assert L.bs_gs_info(None, None, None, None, None) == INVALID
    assert L.bs_gs_degree(None, 16, None) == INVALID
    assert L.bs_ctx_set_tune(None, 0, 0, 4, 16, 0) == INVALID
    assert L.bs_ctx_reset_tune(None) == INVALID
    out = ctypes.c_void_p()
    assert L.bs_gs_create(None, 16, 10, 10, None, ctypes.byref(out)) == INVALID
    assert L.bs_stencil7(None, 0, 3, 0.01, 16, 32, None) == INVALID
    assert L.bs_cg_solve(None, 3, 0.01, 16, 32, 1e-10, 10, None, None) == INVALID
    assert L.bs_cg_ir_solve(None, 1, 3, 0.01, 16, 32, 1e-10, 1e-4, 10, 10, None, None) == INVALID
    assert L.bs_helmholtz_cg_solve(None, 16, 32, 48, 0.01, 64, 80, 1e-10, 10, None, None) == INVALID
    assert L.bs_ctx_create(0, None) == INVALID
    # destroying NULL handles is a no-op
    assert L.bs_ctx_destroy(None) == 0 and L.bs_gs_destroy(None) == 0


def test_mesh_size_limits():
    L = bs.lib
    assert L.bs_mesh_hex_map_host(0, 3, None, None, 16) == 1
    assert L.bs_mesh_hex_map_host(4, 0, None, None, 16) == 1
    assert L.bs_mesh_hex_map_host(4, 3, None, None, None) == 1
    # (K N + 1)^3 must stay below 2^31
    assert L.bs_mesh_hex_map_host(200, 7, None, None, 16) == 1
    assert b"32-bit" in L.bs_last_error()


@pytest.mark.parametrize("K,N,seed", [(1, 1, 0), (2, 1, 1), (3, 2, 2), (4, 3, 3), (3, 7, 4), (2, 15, 5), (8, 3, None)])
def test_host_map_bit_exact_against_oracle(K, N, seed):
    E = K ** 3
    if seed is None:
        perm = orient = None
    else:
        perm = bsgen.permutation(seed, E)
        orient = bsgen.orientations(seed, E)
    got = bs.bs_mesh_hex_map_host(K, N, perm, orient)
    ref = mesh.hex_map(K, N, perm, orient)
    assert got.dtype == np.int32
    assert np.array_equal(got.astype(np.int64), ref)


def test_host_map_rejects_out_of_range_entries():
    perm = np.arange(8, dtype=np.int32)
    perm[3] = 8
    with pytest.raises(bs.BSError):
        bs.bs_mesh_hex_map_host(2, 2, perm, None)
    orient = np.zeros(8, dtype=np.uint8)
    orient[5] = 24
    with pytest.raises(bs.BSError):
        bs.bs_mesh_hex_map_host(2, 2, None, orient)


class _FakeOwner:
    """Stands in for a context or plan: the binding checks tensors before it
    touches the handle, so no device is needed."""
    handle = None
    device = 0
    n_local = n_global = 4

    def expect(self, t, n, what):
        pass


def test_binding_rejects_host_tensors_before_any_launch():
    import torch
    c = _FakeOwner()
    x = torch.zeros(4, dtype=torch.float64)
    y = torch.zeros(4, dtype=torch.float64)
    out = torch.zeros(1, dtype=torch.float64)
    m = torch.zeros(4, dtype=torch.int32)
    calls = [
        lambda: bs.bs_copy(c, x, y),
        lambda: bs.bs_axpy(c, 1.0, x, 1.0, y),
        lambda: bs.bs_norm(c, x, None, out),
        lambda: bs.bs_dot(c, x, y, out),
        lambda: bs.bs_cg_update(c, 1.0, x, y, x.clone(), y.clone(), None, out),
        lambda: bs.bs_axpy_dev(c, x, y, alpha_num=out),
        lambda: bs.bs_cg_update_dev(c, x, y, x.clone(), y.clone(), None, out, alpha_num=out.clone()),
        lambda: bs.bs_gather(c, c, x, y),
        lambda: bs.bs_gs_scatter(c, c, x, y),
        lambda: bs.bs_scatter(c, m, x, y),
        lambda: bs.bs_stencil7(c, 1, 0.01, x[:1], y[:1]),
    ]
    for f in calls:
        with pytest.raises(ValueError, match="HIP device"):
            f()


def test_shipped_tune_table_fits_the_loader():
    """The table bs_ctx_create loads: known operations and dtypes, at most 16 lengths per
    (operation, dtype), ascending lengths, in-range launch shapes (the loader rejects the whole
    table otherwise, and that check needs a device)."""
    path = os.path.join(ROOT, "paper_2009_10917_amd", "tune_gfx950.txt")
    ops = ("copy", "axpy", "norm", "dot", "cg_update", "gather", "scatter", "batch")
    per = {}
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        op, dt, n_min, unroll, cap, variant = f[0], f[1], *map(int, f[2:])
        assert op in ops and dt in ("f64", "f32", "bf16"), line
        assert n_min >= 0 and unroll in (1, 2, 4, 8) and cap >= 1 and 0 <= variant <= 27, line
        assert variant & 3 != 3 and variant & 12 != 12, line
        per.setdefault((op, dt), []).append(n_min)
    assert per
    for key, mins in per.items():
        assert len(mins) <= 16, key
        assert mins == sorted(set(mins)), key
