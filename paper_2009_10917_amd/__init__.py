"""Python binding of the Benchmark-Streaming library (libbs.so, include/bs.h).

Argument marshalling only: every operation runs in the library's HIP kernels
for gfx950.  Vectors are passed as contiguous torch tensors on the current
HIP device (their data pointers go to the C ABI; torch supplies memory and
streams, nothing else).  Each function has the name of the C entry point it
calls, raises ``BSError`` on a non-OK status, and launches on
``torch.cuda.current_stream()`` unless a stream handle is given.

Importing this package fails with ImportError if libbs.so has not been
built (``python paper_2009_10917_amd/build.py``); there is no fallback path.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbs.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "bs.h")

BS_F64, BS_F32, BS_BF16 = 0, 1, 2
STATUS_NAMES = {
    0: "BS_OK", 1: "BS_ERR_INVALID_ARG", 2: "BS_ERR_UNSUPPORTED", 3: "BS_ERR_ALLOC",
    4: "BS_ERR_HIP", 5: "BS_ERR_NO_CONVERGENCE",
}
OP_IDS = {"copy": 0, "axpy": 1, "norm": 2, "dot": 3, "cg_update": 4, "gather": 5, "scatter": 6, "batch": 7}

_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int
_d = ctypes.c_double
_st = ctypes.c_int

# name -> (restype, argtypes), mirroring include/bs.h
PROTOTYPES = {
    "bs_status_string": (ctypes.c_char_p, [_st]),
    "bs_last_error": (ctypes.c_char_p, []),
    "bs_version": (ctypes.c_char_p, []),
    "bs_ctx_create": (_st, [_i32, ctypes.POINTER(_p)]),
    "bs_ctx_destroy": (_st, [_p]),
    "bs_ctx_set_tune": (_st, [_p, _i32, _i32, _i32, _i32, _i32]),
    "bs_ctx_get_tune": (_st, [_p, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "bs_copy": (_st, [_p, _i32, _i64, _p, _p, _p]),
    "bs_axpy": (_st, [_p, _i32, _i64, _d, _p, _d, _p, _p]),
    "bs_norm": (_st, [_p, _i32, _i64, _p, _p, _p, _p]),
    "bs_dot": (_st, [_p, _i32, _i64, _p, _p, _p, _p]),
    "bs_cg_update": (_st, [_p, _i32, _i64, _d, _p, _p, _p, _p, _p, _p, _p]),
    "bs_mesh_hex_map": (_st, [_i64, _i32, _p, _p, _p, _p]),
    "bs_mesh_hex_map_host": (_st, [_i64, _i32, _p, _p, _p]),
    "bs_gs_create": (_st, [_p, _p, _i64, _i64, _p, ctypes.POINTER(_p)]),
    "bs_gs_destroy": (_st, [_p]),
    "bs_gs_info": (_st, [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                         ctypes.POINTER(_i64)]),
    "bs_gs_csr": (_st, [_p, _p, _p, _p]),
    "bs_gs_degree": (_st, [_p, _p, _p]),
    "bs_gs_weights": (_st, [_p, _i32, _p, _p]),
    "bs_gather": (_st, [_p, _p, _i32, _p, _p, _p]),
    "bs_scatter": (_st, [_p, _i32, _i64, _p, _i64, _p, _p, _p]),
    "bs_gs_scatter": (_st, [_p, _p, _i32, _p, _p, _p]),
    "bs_axpy_dev": (_st, [_p, _i32, _i64, _d, _p, _p, _p, _d, _p, _p, _p, _p]),
    "bs_cg_update_dev": (_st, [_p, _i32, _i64, _d, _p, _p, _p, _p, _p, _p, _p, _p, _p]),
    "bs_cg_update_noalloc": (_st, [_i32, _i64, _d, _p, _p, _p, _p, _p, _p, _p]),
    "bs_stencil7": (_st, [_p, _i32, _i64, _d, _p, _p, _p]),
    "bs_elem_create": (_st, [_p, _i32, ctypes.POINTER(_p)]),
    "bs_elem_destroy": (_st, [_p]),
    "bs_elem_rules": (_st, [_p, _p, _p, _p, _p]),
    "bs_helmholtz_local": (_st, [_p, _p, _i64, _p, _i64, _p, _d, _p, _p, _p]),
    "bs_helmholtz_apply": (_st, [_p, _p, _p, _p, _d, _p, _p, _p, _p]),
    "bs_mass_lumped": (_st, [_p, _p, _p, _p, _p, _p, _p]),
    "bs_cg_solve": (_st, [_p, _i64, _d, _p, _p, _d, _i64, _p, _p]),
    "bs_cg_ir_solve": (_st, [_p, _i32, _i64, _d, _p, _p, _d, _d, _i64, _i64, _p, _p]),
    "bs_helmholtz_cg_solve": (_st, [_p, _p, _p, _p, _d, _p, _p, _d, _i64, _p, _p]),
    "bs_mesh_box_map_host": (_st, [_i64, _i32, _p, _p]),
    "bs_gs_order_rows": (_st, [_p, _i64, _i64, _i64, _i32, _i32, _i32, _i32, _p]),
    "bs_gs_order_elements": (_st, [_p, _i64, _p, _i64, _p]),
    "bs_ctx_set_tune_entry": (_st, [_p, _i32, _i32, _i64, _i32, _i32, _i32]),
    "bs_ctx_tune_for": (_st, [_p, _i32, _i32, _i64, _p, _p, _p]),
    "bs_ctx_load_tune": (_st, [_p, ctypes.c_char_p, _p]),
    "bs_ctx_reset_tune": (_st, [_p]),
    "bs_batch_create": (_st, [_p, _i32, _p, _p, _p, _p, _p]),
    "bs_batch_destroy": (_st, [_p]),
    "bs_batch_info": (_st, [_p, _p, _p, _p, _p, _p]),
    "bs_batch_offsets": (_st, [_p, _p, _p]),
    "bs_batch_barrier_timeouts": (_st, [_p, _p, _p]),
    "bs_batch_step": (_st, [_p, _p, _i32, _i32, _p, _d, _d, _p, _p]),
}

BS_BATCH_PER_INSTANCE, BS_BATCH_PER_PHASE, BS_BATCH_PERSISTENT = 0, 1, 2
BATCH_GLOBAL = ("x", "y", "p", "r", "Ap")
BATCH_LOCAL = ("xL", "pL", "wL")
BATCH_SLOTS = ("norm", "dot", "rr", "pAp", "alpha", "rr2", "beta")


class BatchVectors(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in BATCH_GLOBAL + BATCH_LOCAL]


class CgResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("outer_iterations", ctypes.c_int64),
                ("restarts", ctypes.c_int64), ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BSError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {name}" + (f" ({detail})" if detail else ""))


def _load():
    # torch ships its own HIP runtime; loading it first makes libbs bind to
    # that same runtime instead of mapping a second one into the process
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python paper_2009_10917_amd/build.py` "
            "(the streaming operations have no non-HIP implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(status, where):
    if status != 0:
        raise BSError(status, where, lib.bs_last_error().decode())


def _ptr(t, device=None):
    """Device address of a tensor (or an int address, or None).

    Tensors must be contiguous and on a HIP device (the kernels dereference
    the address, so a host tensor is rejected here, before any launch), and
    on `device` when it is given."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError(f"tensors passed to the library must be on a HIP device, not {t.device}")
    if device is not None and t.device.index != device:
        raise ValueError(f"tensor on device {t.device.index}, expected device {device}")
    if not t.is_contiguous():
        raise ValueError("tensors passed to the library must be contiguous")
    return t.data_ptr()


def _ptrs(owner, *ts):
    """Addresses of tensors that must all be on owner's (context or plan) device."""
    return [_ptr(t, owner.device) for t in ts]


def _dtype_id(t):
    import torch
    ids = {torch.float64: BS_F64, torch.float32: BS_F32, torch.bfloat16: BS_BF16}
    if t.dtype not in ids:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return ids[t.dtype]


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _same(a, b, what):
    if a.dtype != b.dtype or a.numel() != b.numel():
        raise ValueError(f"{what}: operands differ in dtype or length")


class Ctx:
    """A bs_ctx handle (one per device and stream)."""

    def __init__(self, handle, device):
        self.handle = handle
        self.device = device

    def close(self):
        if self.handle:
            lib.bs_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A bs_gs gather/scatter plan."""

    def __init__(self, handle, device):
        self.handle = handle
        self.device = device
        self.n_local = self.n_global = self.n_unmasked = self.max_degree = 0

    def expect(self, t, n, what):
        if t is None or t.numel() != n:
            raise ValueError(f"{what}: expected {n} entries")

    def close(self):
        if self.handle:
            lib.bs_gs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bs_version():
    return lib.bs_version().decode()


def bs_ctx_create(device=0):
    h = _p()
    _check(lib.bs_ctx_create(device, ctypes.byref(h)), "bs_ctx_create")
    return Ctx(h.value, device)


def bs_ctx_set_tune(ctx, op, unroll, grid_cap, variant=0, dtype=BS_F64):
    _check(lib.bs_ctx_set_tune(ctx.handle, OP_IDS.get(op, op), dtype, unroll, grid_cap, variant),
           "bs_ctx_set_tune")


def bs_ctx_get_tune(ctx, op, dtype=BS_F64):
    u, g, v = _i32(), _i32(), _i32()
    _check(lib.bs_ctx_get_tune(ctx.handle, OP_IDS.get(op, op), dtype, ctypes.byref(u), ctypes.byref(g),
                               ctypes.byref(v)), "bs_ctx_get_tune")
    return u.value, g.value, v.value


def bs_copy(ctx, x, y, stream=None):
    _same(x, y, "bs_copy")
    px, py = _ptrs(ctx, x, y)
    _check(lib.bs_copy(ctx.handle, _dtype_id(x), x.numel(), px, py, _stream(stream)), "bs_copy")


def bs_axpy(ctx, alpha, x, beta, y, stream=None):
    _same(x, y, "bs_axpy")
    px, py = _ptrs(ctx, x, y)
    _check(lib.bs_axpy(ctx.handle, _dtype_id(x), x.numel(), float(alpha), px, float(beta), py,
                       _stream(stream)), "bs_axpy")


def _out(t, what):
    import torch
    if t is None or t.dtype != torch.float64 or t.numel() < 1:
        raise ValueError(f"{what}: result must go to a float64 device tensor")


def bs_norm(ctx, x, w, out, stream=None):
    _out(out, "bs_norm")
    if w is not None:
        _same(x, w, "bs_norm")
    px, pw, po = _ptrs(ctx, x, w, out)
    _check(lib.bs_norm(ctx.handle, _dtype_id(x), x.numel(), px, pw, po, _stream(stream)), "bs_norm")


def bs_dot(ctx, x, y, out, stream=None):
    _out(out, "bs_dot")
    _same(x, y, "bs_dot")
    px, py, po = _ptrs(ctx, x, y, out)
    _check(lib.bs_dot(ctx.handle, _dtype_id(x), x.numel(), px, py, po, _stream(stream)), "bs_dot")


def bs_cg_update(ctx, alpha, x, p, r, Ap, w, out, stream=None):
    _out(out, "bs_cg_update")
    for v, nm in ((p, "p"), (r, "r"), (Ap, "Ap")):
        _same(x, v, "bs_cg_update " + nm)
    if w is not None:
        _same(x, w, "bs_cg_update w")
    ptrs = _ptrs(ctx, x, p, r, Ap, w, out)
    _check(lib.bs_cg_update(ctx.handle, _dtype_id(x), x.numel(), float(alpha), *ptrs, _stream(stream)),
           "bs_cg_update")


def bs_cg_update_noalloc(alpha, x, p, r, Ap, w, out, stream=None):
    """BS5 without a context: the library's static reduction buffer on the
    current device (calls overlapping on one device race)."""
    import torch
    _out(out, "bs_cg_update_noalloc")
    for v, nm in ((p, "p"), (r, "r"), (Ap, "Ap")):
        _same(x, v, "bs_cg_update_noalloc " + nm)
    if w is not None:
        _same(x, w, "bs_cg_update_noalloc w")
    dev = torch.cuda.current_device()
    ptrs = [_ptr(t, dev) for t in (x, p, r, Ap, w, out)]
    _check(lib.bs_cg_update_noalloc(_dtype_id(x), x.numel(), float(alpha), *ptrs, _stream(stream)),
           "bs_cg_update_noalloc")


def _scalar(t, what):
    """A device binary64 scalar given as a float64 device tensor of one element (or None)."""
    import torch
    if t is None:
        return None
    if t.dtype != torch.float64 or t.numel() != 1:
        raise ValueError(f"{what}: expected a float64 device tensor of one element")
    return t


def bs_axpy_dev(ctx, x, y, alpha=1.0, alpha_num=None, alpha_den=None, beta=1.0, beta_num=None, beta_den=None,
                stream=None):
    """y = a x + b y with a = alpha * (alpha_num / alpha_den) and b = beta * (beta_num / beta_den)
    read on the device (one-element float64 tensors; None reads as 1)."""
    _same(x, y, "bs_axpy_dev")
    sc = [_scalar(t, "bs_axpy_dev") for t in (alpha_num, alpha_den, beta_num, beta_den)]
    px, py, an, ad, bn, bd = _ptrs(ctx, x, y, *sc)
    _check(lib.bs_axpy_dev(ctx.handle, _dtype_id(x), x.numel(), float(alpha), an, ad, px, float(beta), bn, bd, py,
                           _stream(stream)), "bs_axpy_dev")


def bs_cg_update_dev(ctx, x, p, r, Ap, w, out, alpha=1.0, alpha_num=None, alpha_den=None, stream=None):
    """BS5 with alpha = alpha * (alpha_num / alpha_den) read on the device."""
    _out(out, "bs_cg_update_dev")
    for v, nm in ((p, "p"), (r, "r"), (Ap, "Ap")):
        _same(x, v, "bs_cg_update_dev " + nm)
    if w is not None:
        _same(x, w, "bs_cg_update_dev w")
    sc = [_scalar(t, "bs_cg_update_dev") for t in (alpha_num, alpha_den)]
    an, ad, px, pp, pr, pa, pw, po = _ptrs(ctx, *sc, x, p, r, Ap, w, out)
    _check(lib.bs_cg_update_dev(ctx.handle, _dtype_id(x), x.numel(), float(alpha), an, ad, px, pp, pr, pa, pw, po,
                                _stream(stream)), "bs_cg_update_dev")


def bs_mesh_hex_map(K, N, perm, orient, out, stream=None):
    E = K ** 3
    if out.numel() != E * (N + 1) ** 3 or (perm is not None and perm.numel() != E) or \
            (orient is not None and orient.numel() != E):
        raise ValueError("bs_mesh_hex_map: array sizes do not match the mesh")
    _check(lib.bs_mesh_hex_map(K, N, _ptr(perm), _ptr(orient), _ptr(out), _stream(stream)), "bs_mesh_hex_map")


def bs_mesh_hex_map_host(K, N, perm=None, orient=None):
    """Host-side map into a new numpy int32 array (perm int32, orient uint8)."""
    import numpy as np
    n_local = K ** 3 * (N + 1) ** 3
    out = np.empty(n_local, dtype=np.int32)
    pp = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
    oo = None if orient is None else np.ascontiguousarray(orient, dtype=np.uint8)
    _check(lib.bs_mesh_hex_map_host(K, N, None if pp is None else pp.ctypes.data,
                                    None if oo is None else oo.ctypes.data, out.ctypes.data),
           "bs_mesh_hex_map_host")
    return out


def bs_gs_create(ctx, d_map, n_global, stream=None):
    h = _p()
    _check(lib.bs_gs_create(ctx.handle, _ptr(d_map, ctx.device), d_map.numel(), int(n_global), _stream(stream),
                            ctypes.byref(h)), "bs_gs_create")
    plan = Plan(h.value, ctx.device)
    for k, v in bs_gs_info(plan).items():
        setattr(plan, k, v)
    return plan


def bs_gs_info(plan):
    v = [_i64() for _ in range(4)]
    _check(lib.bs_gs_info(plan.handle, *[ctypes.byref(a) for a in v]), "bs_gs_info")
    return dict(zip(("n_local", "n_global", "n_unmasked", "max_degree"), (a.value for a in v)))


def bs_gs_csr(plan, row_starts, col_ids, stream=None):
    plan.expect(row_starts, plan.n_global + 1, "bs_gs_csr row_starts")
    plan.expect(col_ids, plan.n_unmasked, "bs_gs_csr col_ids")
    _check(lib.bs_gs_csr(plan.handle, *_ptrs(plan, row_starts, col_ids), _stream(stream)), "bs_gs_csr")


def bs_gs_degree(plan, deg, stream=None):
    plan.expect(deg, plan.n_global, "bs_gs_degree")
    _check(lib.bs_gs_degree(plan.handle, _ptr(deg, plan.device), _stream(stream)), "bs_gs_degree")


def bs_gs_order_rows(plan, mx, my, mz, tile, box=0, stream=None):
    """Lattice-tiled row order for gather kernel 0 (variants 0, 4, 8; global ids X + mx (Y + my Z)):
    tile^3 blocks, boxes inside a block (box: one side for cubes, or (bx, by, bz);
    0: none)."""
    bx, by, bz = (box, box, box) if isinstance(box, int) else box
    _check(lib.bs_gs_order_rows(plan.handle, int(mx), int(my), int(mz), int(tile), int(bx), int(by), int(bz),
                                _stream(stream)), "bs_gs_order_rows")


def bs_gs_order_elements(plan, nodes_per_element, elem_rank=None, group=1, stream=None):
    """Gather rows and scatter tiles grouped by elements: elem_rank (int32 device tensor, one visiting
    rank per element) or, when None, an order the library derives from the map's connectivity;
    `group` elements of consecutive ranks are visited together."""
    import torch
    if elem_rank is not None:
        if elem_rank.dtype != torch.int32 or elem_rank.numel() != plan.n_local // int(nodes_per_element):
            raise ValueError("bs_gs_order_elements: elem_rank must be int32 with one entry per element")
    _check(lib.bs_gs_order_elements(plan.handle, int(nodes_per_element), _ptr(elem_rank, plan.device), int(group),
                                    _stream(stream)), "bs_gs_order_elements")


def bs_gs_weights(plan, wL, stream=None):
    plan.expect(wL, plan.n_local, "bs_gs_weights")
    _check(lib.bs_gs_weights(plan.handle, _dtype_id(wL), _ptr(wL, plan.device), _stream(stream)), "bs_gs_weights")


def bs_gather(ctx, plan, xL, xG, stream=None):
    plan.expect(xL, plan.n_local, "bs_gather xL")
    plan.expect(xG, plan.n_global, "bs_gather xG")
    pl, pg = _ptrs(plan, xL, xG)
    _check(lib.bs_gather(ctx.handle, plan.handle, _dtype_id(xL), pl, pg, _stream(stream)), "bs_gather")


def bs_gs_scatter(ctx, plan, xG, xL, stream=None):
    plan.expect(xL, plan.n_local, "bs_gs_scatter xL")
    plan.expect(xG, plan.n_global, "bs_gs_scatter xG")
    pg, pl = _ptrs(plan, xG, xL)
    _check(lib.bs_gs_scatter(ctx.handle, plan.handle, _dtype_id(xG), pg, pl, _stream(stream)), "bs_gs_scatter")


def bs_scatter(ctx, d_map, xG, xL, stream=None):
    """x_L[l] = x_G[d_map[l]] for ids in [0, len(xG)); other entries of xL untouched."""
    import torch
    if d_map.dtype != torch.int32 or d_map.numel() != xL.numel() or xG.dtype != xL.dtype:
        raise ValueError("bs_scatter: map must be int32 with one entry per local value, xG and xL one dtype")
    pm, pg, pl = _ptrs(ctx, d_map, xG, xL)
    _check(lib.bs_scatter(ctx.handle, _dtype_id(xG), xL.numel(), pm, xG.numel(), pg, pl, _stream(stream)),
           "bs_scatter")


def bs_stencil7(ctx, m, shift, x, y, stream=None):
    _same(x, y, "bs_stencil7")
    if x.numel() != m ** 3:
        raise ValueError("bs_stencil7: vectors must have m^3 entries")
    _check(lib.bs_stencil7(ctx.handle, _dtype_id(x), m, float(shift), *_ptrs(ctx, x, y), _stream(stream)),
           "bs_stencil7")


# ---------------------------------------------------------------- element operators

class Elem:
    """A bs_elem: the 1D rules and basis tables of degree N."""

    def __init__(self, handle, device, N):
        self.handle = handle
        self.device = device
        self.N = N
        self.P = (N + 1) ** 3

    def close(self):
        if self.handle:
            lib.bs_elem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bs_elem_create(ctx, N):
    h = _p()
    _check(lib.bs_elem_create(ctx.handle, int(N), ctypes.byref(h)), "bs_elem_create")
    return Elem(h.value, ctx.device, int(N))


def bs_elem_rules(el):
    """(gll_x, gll_w, gauss_x, gauss_w) as numpy arrays of N+1 values."""
    import numpy as np
    out = [np.empty(el.N + 1) for _ in range(4)]
    _check(lib.bs_elem_rules(el.handle, *[a.ctypes.data for a in out]), "bs_elem_rules")
    return tuple(out)


def _f64(t, n, what):
    import torch
    if t is None or t.dtype != torch.float64 or t.numel() != n:
        raise ValueError(f"{what}: expected a float64 device tensor of {n} entries")


def bs_helmholtz_local(ctx, el, d_map, geo, lam, xG, yL, stream=None):
    """y_L = A_L Z x_G for the elements of d_map (int32, n_elem (N+1)^3 entries)."""
    import torch
    if d_map.dtype != torch.int32 or d_map.numel() % el.P:
        raise ValueError("bs_helmholtz_local: map must be int32 with whole elements")
    E = d_map.numel() // el.P
    _f64(geo, 7 * E, "bs_helmholtz_local geo")
    _f64(yL, E * el.P, "bs_helmholtz_local yL")
    _f64(xG, xG.numel(), "bs_helmholtz_local xG")
    pm, pg, px, py = _ptrs(ctx, d_map, geo, xG, yL)
    _check(lib.bs_helmholtz_local(ctx.handle, el.handle, E, pm, xG.numel(), pg, float(lam), px, py,
                                  _stream(stream)), "bs_helmholtz_local")


def bs_helmholtz_apply(ctx, el, plan, geo, lam, xG, yL_work, yG, stream=None):
    _f64(geo, 7 * (plan.n_local // el.P), "bs_helmholtz_apply geo")
    _f64(xG, plan.n_global, "bs_helmholtz_apply xG")
    _f64(yG, plan.n_global, "bs_helmholtz_apply yG")
    _f64(yL_work, plan.n_local, "bs_helmholtz_apply yL_work")
    pg, px, pw, py = _ptrs(ctx, geo, xG, yL_work, yG)
    _check(lib.bs_helmholtz_apply(ctx.handle, el.handle, plan.handle, pg, float(lam), px, pw, py, _stream(stream)),
           "bs_helmholtz_apply")


def bs_mass_lumped(ctx, el, plan, geo, xG, yG, stream=None):
    _f64(geo, 7 * (plan.n_local // el.P), "bs_mass_lumped geo")
    _f64(xG, plan.n_global, "bs_mass_lumped xG")
    _f64(yG, plan.n_global, "bs_mass_lumped yG")
    pg, px, py = _ptrs(ctx, geo, xG, yG)
    _check(lib.bs_mass_lumped(ctx.handle, el.handle, plan.handle, pg, px, py, _stream(stream)), "bs_mass_lumped")


def _solver_vectors(m, b, x, what):
    import torch
    for v in (b, x):
        if v.dtype != torch.float64 or v.numel() != m ** 3:
            raise ValueError(f"{what}: b and x must be float64 with m^3 entries")


def bs_cg_solve(ctx, m, shift, b, x, tol=1e-10, max_iter=100000, stream=None, check=True):
    """Binary64 CG on the 7-point operator; returns the result record as a dict."""
    _solver_vectors(m, b, x, "bs_cg_solve")
    res = CgResult()
    st = lib.bs_cg_solve(ctx.handle, m, float(shift), *_ptrs(ctx, b, x), float(tol), int(max_iter),
                         ctypes.byref(res), _stream(stream))
    if check:
        _check(st, "bs_cg_solve")
    out = res.as_dict()
    out["status"] = STATUS_NAMES.get(st, st)
    return out


def bs_helmholtz_cg_solve(ctx, el, plan, geo, lam, b, x, tol=1e-10, max_iter=100000, stream=None, check=True):
    """Binary64 CG on the assembled Helmholtz operator Z^T A_L Z of the plan's
    map; x is the starting guess, overwritten.  Returns the result record."""
    _f64(geo, 7 * (plan.n_local // el.P), "bs_helmholtz_cg_solve geo")
    _f64(b, plan.n_global, "bs_helmholtz_cg_solve b")
    _f64(x, plan.n_global, "bs_helmholtz_cg_solve x")
    res = CgResult()
    st = lib.bs_helmholtz_cg_solve(ctx.handle, el.handle, plan.handle, *_ptrs(ctx, geo), float(lam),
                                   *_ptrs(ctx, b, x), float(tol), int(max_iter), ctypes.byref(res), _stream(stream))
    if check:
        _check(st, "bs_helmholtz_cg_solve")
    out = res.as_dict()
    out["status"] = STATUS_NAMES.get(st, st)
    return out


def bs_cg_ir_solve(ctx, inner_dtype, m, shift, b, x, tol=1e-10, inner_tol=1e-4, max_inner=400, max_outer=50,
                   stream=None, check=True):
    """Mixed-precision iterative refinement; inner_dtype is BS_F32, BS_BF16 or BS_F64."""
    _solver_vectors(m, b, x, "bs_cg_ir_solve")
    res = CgResult()
    st = lib.bs_cg_ir_solve(ctx.handle, int(inner_dtype), m, float(shift), *_ptrs(ctx, b, x), float(tol),
                            float(inner_tol), int(max_inner), int(max_outer), ctypes.byref(res), _stream(stream))
    if check:
        _check(st, "bs_cg_ir_solve")
    out = res.as_dict()
    out["status"] = STATUS_NAMES.get(st, st)
    return out


# ---------------------------------------------------------------- batched instances

def bs_mesh_box_map_host(E, N):
    """Box mesh of E elements at degree N: (int32 numpy map, n_global)."""
    import numpy as np
    out = np.empty(int(E) * (int(N) + 1) ** 3, dtype=np.int32)
    ng = _i64()
    _check(lib.bs_mesh_box_map_host(int(E), int(N), out.ctypes.data, ctypes.byref(ng)), "bs_mesh_box_map_host")
    return out, ng.value


class Batch:
    """A bs_batch: instance sizes, offsets and the block-diagonal plan."""

    def __init__(self, handle, n_inst):
        self.handle = handle
        self.n_inst = n_inst

    def close(self):
        if self.handle:
            lib.bs_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bs_batch_create(ctx, n_local, n_global, d_map, stream=None):
    import numpy as np
    nl = np.ascontiguousarray(n_local, dtype=np.int64)
    ng = np.ascontiguousarray(n_global, dtype=np.int64)
    if nl.size != ng.size or d_map.numel() != int(nl.sum()):
        raise ValueError("bs_batch_create: sizes and map disagree")
    h = _p()
    _check(lib.bs_batch_create(ctx.handle, int(nl.size), nl.ctypes.data, ng.ctypes.data, _ptr(d_map, ctx.device),
                               _stream(stream), ctypes.byref(h)), "bs_batch_create")
    b = Batch(h.value, int(nl.size))
    v = [_i64() for _ in range(4)] + [ctypes.c_int32()]
    _check(lib.bs_batch_info(b.handle, *[ctypes.byref(a) for a in v]), "bs_batch_info")
    b.n_local, b.n_global, b.n_chunks_local, b.n_chunks_global, b.persistent_blocks = (a.value for a in v)
    b.off_local = np.empty(b.n_inst + 1, dtype=np.int64)
    b.off_global = np.empty(b.n_inst + 1, dtype=np.int64)
    _check(lib.bs_batch_offsets(b.handle, b.off_local.ctypes.data, b.off_global.ctypes.data), "bs_batch_offsets")
    return b


def bs_batch_barrier_timeouts(batch, stream=None):
    c = ctypes.c_int32()
    _check(lib.bs_batch_barrier_timeouts(batch.handle, ctypes.byref(c), _stream(stream)), "bs_batch_barrier_timeouts")
    return c.value


def bs_batch_step(ctx, batch, vectors, alpha, beta, out, mode=BS_BATCH_PER_PHASE, stream=None):
    """One batch step; vectors maps x, y, p, r, Ap, xL, pL, wL to tensors of one dtype."""
    dt = None
    for k in BATCH_GLOBAL + BATCH_LOCAL:
        t = vectors[k]
        n = batch.n_global if k in BATCH_GLOBAL else batch.n_local
        if t.numel() != n:
            raise ValueError(f"bs_batch_step: {k} needs {n} entries")
        d = _dtype_id(t)
        if dt is not None and d != dt:
            raise ValueError("bs_batch_step: vectors differ in dtype")
        dt = d
    _out(out, "bs_batch_step")
    if out.numel() < 8 * batch.n_inst:
        raise ValueError("bs_batch_step: out needs 8 doubles per instance")
    v = BatchVectors(*_ptrs(ctx, *[vectors[k] for k in BATCH_GLOBAL + BATCH_LOCAL]))
    _check(lib.bs_batch_step(ctx.handle, batch.handle, dt, int(mode), ctypes.byref(v), float(alpha), float(beta),
                             _ptr(out, ctx.device), _stream(stream)), "bs_batch_step")


# ---------------------------------------------------------------- tune tables

def _op_id(op):
    return OP_IDS[op] if isinstance(op, str) else int(op)


def bs_ctx_set_tune_entry(ctx, op, n_min, unroll, grid_cap, variant=0, dtype=BS_F64):
    _check(lib.bs_ctx_set_tune_entry(ctx.handle, _op_id(op), int(dtype), int(n_min), int(unroll), int(grid_cap),
                                     int(variant)), "bs_ctx_set_tune_entry")


def bs_ctx_tune_for(ctx, op, n, dtype=BS_F64):
    v = [ctypes.c_int() for _ in range(3)]
    _check(lib.bs_ctx_tune_for(ctx.handle, _op_id(op), int(dtype), int(n), *[ctypes.byref(a) for a in v]),
           "bs_ctx_tune_for")
    return tuple(a.value for a in v)


def bs_ctx_reset_tune(ctx):
    """Restore the tune table the context was created with (defaults, then the installed table)."""
    _check(lib.bs_ctx_reset_tune(ctx.handle), "bs_ctx_reset_tune")


def bs_ctx_load_tune(ctx, path):
    n = ctypes.c_int()
    _check(lib.bs_ctx_load_tune(ctx.handle, str(path).encode(), ctypes.byref(n)), "bs_ctx_load_tune")
    return n.value
