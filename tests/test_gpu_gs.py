"""GPU parity of the mesh map, the gather/scatter plan, BS6 and BS7.

Map, CSR, degrees, weights, gather and scatter are all compared bit for bit
with the oracle (gather adds in the oracle's fixed order, so its bits are
reproducible; the stated bar is 1e-14 relative).
"""

import numpy as np
import pytest
import torch

import bsgen
from oracle import mesh, ops

pytestmark = pytest.mark.gpu

import paper_2009_10917_amd as bs  # noqa: E402
from gpu_util import bits, dev_uniform, host_uniform, to_host  # noqa: E402

# kernel choice, plus 4 = dispatch order, plus 8 = XCD runs of 256 blocks; plus 16 = cached accesses (kernel 0)
VARIANTS = [0, 1, 2, 4, 5, 6, 8, 9, 10, 16, 20, 24]
MESHES = [(1, 1, None), (2, 1, 1), (3, 2, 2), (8, 3, None), (4, 7, 3), (3, 15, 4), (6, 5, 5), (5, 4, None),
          (12, 2, 6)]


def with_variant(ctx, variant, unroll=4):
    bs.bs_ctx_set_tune(ctx, "gather", 1, 1 << 30, variant)
    bs.bs_ctx_set_tune(ctx, "scatter", unroll, 1 << 30, variant)


@pytest.fixture
def ctx():
    # a context per test: tests set one launch shape for every length, which
    # would otherwise replace the shared context's whole tune table
    c = bs.bs_ctx_create(0)
    yield c
    c.close()


def device_map(K, N, seed):
    E = K ** 3
    if seed is None:
        perm = orient = None
        dp = do = None
    else:
        perm = bsgen.permutation(seed, E)
        orient = bsgen.orientations(seed, E)
        dp = torch.from_numpy(perm.astype(np.int32)).cuda()
        do = torch.from_numpy(orient.astype(np.uint8)).cuda()
    d_map = torch.empty(E * (N + 1) ** 3, dtype=torch.int32, device="cuda")
    bs.bs_mesh_hex_map(K, N, dp, do, d_map)
    return d_map, mesh.hex_map(K, N, perm, orient)


@pytest.mark.parametrize("K,N,seed", MESHES)
def test_map_plan_gather_scatter(ctx, K, N, seed):
    E, NL, NG = mesh.sizes(K, N)
    d_map, ref_map = device_map(K, N, seed)
    assert np.array_equal(to_host(d_map).astype(np.int64), ref_map)
    plan = bs.bs_gs_create(ctx, d_map, NG)
    assert (plan.n_local, plan.n_global, plan.n_unmasked) == (NL, NG, NL)
    rs_ref, ci_ref = mesh.csr_inverse(ref_map, NG)
    deg_ref = mesh.degree(ref_map, NG)
    assert plan.max_degree == int(deg_ref.max())
    rs = torch.empty(NG + 1, dtype=torch.int32, device="cuda")
    ci = torch.empty(NL, dtype=torch.int32, device="cuda")
    bs.bs_gs_csr(plan, rs, ci)
    assert np.array_equal(to_host(rs), rs_ref) and np.array_equal(to_host(ci), ci_ref)
    deg = torch.empty(NG, dtype=torch.int32, device="cuda")
    bs.bs_gs_degree(plan, deg)
    assert np.array_equal(to_host(deg), deg_ref)
    w_ref = mesh.weights(ref_map, NG)
    for dt in (torch.float64, torch.float32, torch.bfloat16):
        w = torch.empty(NL, dtype=dt, device="cuda")
        bs.bs_gs_weights(plan, w)
        if dt == torch.float64:
            assert np.array_equal(bits(to_host(w)), bits(w_ref))
        elif dt == torch.float32:
            assert np.array_equal(to_host(w), bsgen.round_f32(w_ref))
        else:
            assert np.array_equal(to_host(w), bsgen.round_bf16_bits(w_ref))
    # BS6 gather and BS7 scatter, both kernel variants
    g_ref = ops.gather(rs_ref, ci_ref, host_uniform(NL, 11))
    s_ref = ops.scatter(ref_map, host_uniform(NG, 12), host_uniform(NL, 11))
    for variant in VARIANTS:
        with_variant(ctx, variant)
        xL = dev_uniform(NL, 11)
        xG = torch.full((NG,), float("nan"), dtype=torch.float64, device="cuda")
        bs.bs_gather(ctx, plan, xL, xG)
        assert np.array_equal(bits(to_host(xG)), bits(g_ref)), variant
        xG2 = dev_uniform(NG, 12)
        bs.bs_gs_scatter(ctx, plan, xG2, xL)
        assert np.array_equal(bits(to_host(xL)), bits(s_ref)), variant
    # gather(scatter(1)) is the degree, exactly
    ones = torch.ones(NG, dtype=torch.float64, device="cuda")
    bs.bs_gs_scatter(ctx, plan, ones, xL)
    bs.bs_gather(ctx, plan, xL, xG)
    assert np.array_equal(to_host(xG), deg_ref.astype(np.float64))
    plan.close()


@pytest.mark.parametrize("variant", VARIANTS)
def test_masked_entries(ctx, variant):
    with_variant(ctx, variant)
    K, N = 5, 3
    E, NL, NG = mesh.sizes(K, N)
    ref_map = mesh.hex_map(K, N, bsgen.permutation(9, E), bsgen.orientations(9, E))
    ref_map[::7] = -1
    ref_map[3::11] = -5
    d_map = torch.from_numpy(ref_map.astype(np.int32)).cuda()
    plan = bs.bs_gs_create(ctx, d_map, NG)
    assert plan.n_unmasked == int(np.count_nonzero(ref_map >= 0))
    rs_ref, ci_ref = mesh.csr_inverse(ref_map, NG)
    xL = dev_uniform(NL, 11)
    xG = torch.empty(NG, dtype=torch.float64, device="cuda")
    bs.bs_gather(ctx, plan, xL, xG)
    assert np.array_equal(bits(to_host(xG)), bits(ops.gather(rs_ref, ci_ref, host_uniform(NL, 11))))
    xG2 = dev_uniform(NG, 12)
    bs.bs_gs_scatter(ctx, plan, xG2, xL)
    assert np.array_equal(bits(to_host(xL)), bits(ops.scatter(ref_map, host_uniform(NG, 12), host_uniform(NL, 11))))
    w = torch.empty(NL, dtype=torch.float64, device="cuda")
    bs.bs_gs_weights(plan, w)
    assert np.array_equal(bits(to_host(w)), bits(mesh.weights(ref_map, NG)))


@pytest.mark.parametrize("variant", VARIANTS)
def test_high_degree_rows_use_the_unstaged_path(ctx, variant):
    with_variant(ctx, variant)
    # 7 global nodes with ~14000 copies each: a workgroup's rows hold far
    # more values than its LDS stage, so the direct path adds them
    NL, NG = 100_003, 7
    ref_map = (np.arange(NL) * 5) % NG
    ref_map[::13] = -1
    d_map = torch.from_numpy(ref_map.astype(np.int32)).cuda()
    plan = bs.bs_gs_create(ctx, d_map, NG)
    assert plan.max_degree > 10000
    rs_ref, ci_ref = mesh.csr_inverse(ref_map, NG)
    xL = dev_uniform(NL, 11)
    xG = torch.empty(NG, dtype=torch.float64, device="cuda")
    bs.bs_gather(ctx, plan, xL, xG)
    assert np.array_equal(bits(to_host(xG)), bits(ops.gather(rs_ref, ci_ref, host_uniform(NL, 11))))


@pytest.mark.parametrize("variant", VARIANTS)
def test_rows_without_copies_and_empty_plans(ctx, variant):
    with_variant(ctx, variant)
    # global ids 0..9, only even ones used: odd rows gather to +0.0
    ref_map = np.array([0, 2, 2, 4, 6, 8, 8, 8, -1], dtype=np.int64)
    plan = bs.bs_gs_create(ctx, torch.from_numpy(ref_map.astype(np.int32)).cuda(), 10)
    xL = torch.tensor([1.0, -0.0, -0.0, 3.0, 4.0, 5.0, 6.0, 7.0, 9.0], dtype=torch.float64, device="cuda")
    xG = torch.full((10,), -1.0, dtype=torch.float64, device="cuda")
    bs.bs_gather(ctx, plan, xL, xG)
    got = to_host(xG)
    assert list(got) == [1.0, 0.0, 0.0, 0.0, 3.0, 0.0, 4.0, 0.0, 18.0, 0.0]
    assert not np.any(np.signbit(got))
    empty = bs.bs_gs_create(ctx, torch.empty(0, dtype=torch.int32, device="cuda"), 5)
    assert empty.n_unmasked == 0
    xG = torch.full((5,), 7.0, dtype=torch.float64, device="cuda")
    bs.bs_gather(ctx, empty, torch.empty(0, dtype=torch.float64, device="cuda"), xG)
    assert np.array_equal(to_host(xG), np.zeros(5))


def test_invalid_maps_and_meshes_are_rejected(ctx):
    bad = torch.tensor([0, 1, 5], dtype=torch.int32, device="cuda")
    with pytest.raises(bs.BSError) as e:
        bs.bs_gs_create(ctx, bad, 5)
    assert e.value.status == 1
    perm = torch.arange(8, dtype=torch.int32, device="cuda")
    orient = torch.zeros(8, dtype=torch.uint8, device="cuda")
    orient[3] = 30
    out = torch.empty(8 * 27, dtype=torch.int32, device="cuda")
    with pytest.raises(bs.BSError):
        bs.bs_mesh_hex_map(2, 2, perm, orient, out)
    with pytest.raises(ValueError):
        plan = bs.bs_gs_create(ctx, torch.tensor([0, 1], dtype=torch.int32, device="cuda"), 2)
        bs.bs_gather(ctx, plan, torch.zeros(3, dtype=torch.float64, device="cuda"),
                     torch.zeros(2, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("unroll", [1, 2, 4, 8])
def test_scatter_map_order_unrolls(ctx, unroll):
    K, N = 7, 4
    E, NL, NG = mesh.sizes(K, N)
    d_map, ref_map = device_map(K, N, 31)
    plan = bs.bs_gs_create(ctx, d_map, NG)
    with_variant(ctx, 2, unroll=unroll)
    xL = dev_uniform(NL, 11)
    bs.bs_gs_scatter(ctx, plan, dev_uniform(NG, 12), xL)
    ref = ops.scatter(ref_map, host_uniform(NG, 12), host_uniform(NL, 11))
    assert np.array_equal(bits(to_host(xL)), bits(ref))


@pytest.mark.parametrize("variant", [0, 1, 4, 5, 8, 9, 16, 24])
@pytest.mark.parametrize("tpw", [1, 2, 4, 8])
def test_scatter_tiles_per_workgroup(ctx, variant, tpw):
    # tile variants take 1, 2 or 4 tiles of the visiting order per workgroup
    # (the tune entry's unroll; 8 rounds down to 4); 7^3 elements of degree 3
    # give 7^3/8 = 42.9 tiles, so the last workgroup holds a partial tile and
    # missing ones
    K, N = 7, 3
    E, NL, NG = mesh.sizes(K, N)
    _, ref_map = device_map(K, N, 13)
    ref_map = ref_map.copy()
    ref_map[5::9] = -1
    plan = bs.bs_gs_create(ctx, torch.from_numpy(ref_map.astype(np.int32)).cuda(), NG)
    bs.bs_ctx_set_tune(ctx, "scatter", tpw, 1 << 30, variant)
    xL = dev_uniform(NL, 11)
    bs.bs_gs_scatter(ctx, plan, dev_uniform(NG, 12), xL)
    ref = ops.scatter(ref_map, host_uniform(NG, 12), host_uniform(NL, 11))
    assert np.array_equal(bits(to_host(xL)), bits(ref))


@pytest.mark.parametrize("tpw", [1, 2, 4])
def test_scatter_sorted_tiles_with_wide_id_spans(ctx, tpw):
    # ids spread over 2^24 global entries: tiles span more than 2^23 ids, so
    # the plan keeps (id, offset) pairs instead of packed words
    rng = np.random.default_rng(5)
    NG, NL = (1 << 24) + 3, 5000
    ref_map = rng.integers(0, NG, NL).astype(np.int64)
    ref_map[::11] = -1
    plan = bs.bs_gs_create(ctx, torch.from_numpy(ref_map.astype(np.int32)).cuda(), NG)
    bs.bs_ctx_set_tune(ctx, "scatter", tpw, 1 << 30, 0)
    xL = dev_uniform(NL, 11)
    bs.bs_gs_scatter(ctx, plan, dev_uniform(NG, 12), xL)
    ref = ops.scatter(ref_map, host_uniform(NG, 12), host_uniform(NL, 11))
    assert np.array_equal(bits(to_host(xL)), bits(ref))


def test_scatter_with_no_global_entries(ctx):
    # every local entry masked: nothing is written, whatever the variant
    ref_map = np.full(1000, -1, dtype=np.int32)
    plan = bs.bs_gs_create(ctx, torch.from_numpy(ref_map).cuda(), 0)
    for variant in (0, 1, 2):
        bs.bs_ctx_set_tune(ctx, "scatter", 4, 1 << 30, variant)
        xL = torch.full((1000,), 3.0, dtype=torch.float64, device="cuda")
        bs.bs_gs_scatter(ctx, plan, torch.empty(0, dtype=torch.float64, device="cuda"), xL)
        assert np.array_equal(to_host(xL), np.full(1000, 3.0))


def test_many_empty_rows_and_long_rows(ctx):
    # globals with no copies between used ones, plus a few very long rows:
    # exercises blocks with many rows and windows that rows overrun
    rng = np.random.default_rng(3)
    NG = 200_000
    used = np.sort(rng.choice(NG, 3000, replace=False))
    ref_map = used[rng.integers(0, used.size, 60_000)]
    ref_map[rng.integers(0, 60_000, 5000)] = used[7]      # one row of degree ~5000
    ref_map[rng.integers(0, 60_000, 3000)] = used[-1]
    plan = bs.bs_gs_create(ctx, torch.from_numpy(ref_map.astype(np.int32)).cuda(), NG)
    rs_ref, ci_ref = mesh.csr_inverse(ref_map, NG)
    xLh = bsgen.uniform(1, 11, ref_map.size)
    ref = ops.gather(rs_ref, ci_ref, xLh)
    for variant in VARIANTS:
        with_variant(ctx, variant)
        xG = torch.full((NG,), float("nan"), dtype=torch.float64, device="cuda")
        bs.bs_gather(ctx, plan, torch.from_numpy(xLh).cuda(), xG)
        assert np.array_equal(bits(to_host(xG)), bits(ref)), variant


@pytest.mark.parametrize("tile,sub", [(0, 0), (1000, 0), (1000, 37)])
def test_gather_windows_near_the_stage_size(ctx, tile, sub):
    # degrees 1..255 (the largest the permuted order takes), local copies in
    # random order: windows of up to chunk + 254 = 2047 values, each loaded in
    # address order and put back in CSR order; rows still add copies in
    # ascending local index.  tile > 0 re-orders rows on a 1-D lattice.
    rng = np.random.default_rng(17)
    NG = 5000
    deg = rng.integers(1, 256, NG)
    deg[[0, 1, 2, NG // 2, NG - 1]] = 255
    deg[rng.choice(NG, 300, replace=False)] = 0  # rows without copies
    ref_map = rng.permutation(np.repeat(np.arange(NG), deg))
    plan = bs.bs_gs_create(ctx, torch.from_numpy(ref_map.astype(np.int32)).cuda(), NG)
    assert plan.max_degree == 255
    if tile:
        bs.bs_gs_order_rows(plan, NG, 1, 1, tile, sub)
    rs_ref, ci_ref = mesh.csr_inverse(ref_map, NG)
    xLh = bsgen.uniform(2, 11, ref_map.size)
    ref = ops.gather(rs_ref, ci_ref, xLh)
    with_variant(ctx, 0)
    xG = torch.full((NG,), float("nan"), dtype=torch.float64, device="cuda")
    bs.bs_gather(ctx, plan, torch.from_numpy(xLh).cuda(), xG)
    assert np.array_equal(bits(to_host(xG)), bits(ref))


def test_gather_permuted_order_up_to_degree_1024(ctx):
    # rows of degree up to 1024 keep the permuted order (windows of up to
    # 1023 + 1024 entries); one row more than that and variant 0 falls back
    # to the global order; both give the definition's bits
    rng = np.random.default_rng(23)
    NG = 3000
    deg = rng.integers(1, 9, NG)
    deg[[5, 1700, NG - 1]] = 1024
    deg[[6, 7]] = [1000, 999]
    for extra in (0, 1):
        d = deg.copy()
        d[5] += extra
        ref_map = rng.permutation(np.repeat(np.arange(NG), d))
        plan = bs.bs_gs_create(ctx, torch.from_numpy(ref_map.astype(np.int32)).cuda(), NG)
        assert plan.max_degree == 1024 + extra
        if extra == 0:
            bs.bs_gs_order_rows(plan, NG, 1, 1, 64, 0)
        else:
            with pytest.raises(bs.BSError):
                bs.bs_gs_order_rows(plan, NG, 1, 1, 64, 0)
        rs_ref, ci_ref = mesh.csr_inverse(ref_map, NG)
        xLh = bsgen.uniform(3, 11, ref_map.size)
        with_variant(ctx, 0)
        xG = torch.full((NG,), float("nan"), dtype=torch.float64, device="cuda")
        bs.bs_gather(ctx, plan, torch.from_numpy(xLh).cuda(), xG)
        assert np.array_equal(bits(to_host(xG)), bits(ops.gather(rs_ref, ci_ref, xLh)))


def test_gather_scatter_deterministic(ctx):
    K, N = 10, 7
    E, NL, NG = mesh.sizes(K, N)
    d_map, _ = device_map(K, N, 21)
    plan = bs.bs_gs_create(ctx, d_map, NG)
    xL = dev_uniform(NL, 11)
    outs = []
    for _ in range(3):
        xG = torch.empty(NG, dtype=torch.float64, device="cuda")
        bs.bs_gather(ctx, plan, xL, xG)
        outs.append(bits(to_host(xG)))
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


@pytest.mark.parametrize("remap", [0, 4])
@pytest.mark.parametrize("K,N,tile,box", [(6, 5, 1, 0), (6, 5, 4, 0), (7, 3, 7, 0), (5, 7, 64, 0), (9, 2, 5, 0),
                                          (6, 5, 10, 5), (7, 3, 12, 6), (5, 7, 28, 14), (9, 2, 7, 3), (6, 7, 98, 14),
                                          (4, 7, 5, 9), (6, 7, 42, (42, 7, 7)), (5, 3, 12, (12, 3, 6)),
                                          (7, 4, 16, (0, 4, 8)), (5, 5, 11, (2, 3, 4))])
def test_gather_lattice_tiled_order(ctx, K, N, tile, box, remap):
    # the tiled row order changes which rows a workgroup adds, not how a row is summed
    E, NL, NG = mesh.sizes(K, N)
    d_map, ids = device_map(K, N, 5)
    plan = bs.bs_gs_create(ctx, d_map, NG)
    M = K * N + 1
    bs.bs_gs_order_rows(plan, M, M, M, tile, box)
    with_variant(ctx, 0 + remap)
    xL = dev_uniform(NL, 11)
    xG = torch.empty(NG, dtype=torch.float64, device="cuda")
    bs.bs_gather(ctx, plan, xL, xG)
    rs, ci = mesh.csr_inverse(ids, NG)
    assert np.array_equal(bits(to_host(xG)), bits(ops.gather(rs, ci, to_host(xL))))


def test_gather_lattice_order_masked_and_errors(ctx):
    K, N = 5, 4
    E, NL, NG = mesh.sizes(K, N)
    d_map, ids = device_map(K, N, 9)
    ids = ids.copy()
    ids[::7] = -1  # masked copies; some rows lose every copy
    ids[ids == 17] = -1
    plan = bs.bs_gs_create(ctx, torch.from_numpy(ids.astype(np.int32)).cuda(), NG)
    M = K * N + 1
    with pytest.raises(bs.BSError):
        bs.bs_gs_order_rows(plan, M, M, M + 1, 4)
    with pytest.raises(bs.BSError):
        bs.bs_gs_order_rows(plan, M, M, M, 0)
    with pytest.raises(bs.BSError):
        bs.bs_gs_order_rows(plan, M, M, M, 4, -1)
    with pytest.raises(bs.BSError):
        bs.bs_gs_order_rows(plan, M, M, M, 4, (0, -2, 0))
    with pytest.raises(bs.BSError):
        bs.bs_gs_order_rows(plan, M, M, M, 1 << 30, 1)  # more boxes than 32-bit keys hold
    bs.bs_gs_order_rows(plan, M, M, M, 3, 2)
    with_variant(ctx, 0)
    xL = dev_uniform(NL, 11)
    xG = torch.full((NG,), 7.0, dtype=torch.float64, device="cuda")
    bs.bs_gather(ctx, plan, xL, xG)
    rs, ci = mesh.csr_inverse(ids, NG)
    assert np.array_equal(bits(to_host(xG)), bits(ops.gather(rs, ci, to_host(xL))))


@pytest.mark.parametrize("remap", [0, 8])
@pytest.mark.parametrize("K,N,seed,group", [(1, 1, None, 1), (3, 2, 2, 1), (4, 7, 3, 1), (6, 5, 5, 7), (8, 3, None, 64),
                                            (5, 4, 7, 1000), (3, 15, 4, 2)])
def test_gather_element_order_derived(ctx, K, N, seed, group, remap):
    # the order derived from the map's connectivity changes which rows a
    # workgroup adds, not how a row is summed
    E, NL, NG = mesh.sizes(K, N)
    d_map, ids = device_map(K, N, seed)
    plan = bs.bs_gs_create(ctx, d_map, NG)
    bs.bs_gs_order_elements(plan, (N + 1) ** 3, None, group)
    with_variant(ctx, 0 + remap)
    xL = dev_uniform(NL, 11)
    xG = torch.empty(NG, dtype=torch.float64, device="cuda")
    bs.bs_gather(ctx, plan, xL, xG)
    rs, ci = mesh.csr_inverse(ids, NG)
    assert np.array_equal(bits(to_host(xG)), bits(ops.gather(rs, ci, to_host(xL))))


@pytest.mark.parametrize("ranks", ["reversed", "random", "constant"])
def test_gather_element_order_given_and_masked(ctx, ranks):
    K, N = 5, 4
    E, NL, NG = mesh.sizes(K, N)
    _, ids = device_map(K, N, 9)
    ids = ids.copy()
    ids[::7] = -1  # masked copies, masked corners; some rows lose every copy
    ids[ids == 17] = -1
    plan = bs.bs_gs_create(ctx, torch.from_numpy(ids.astype(np.int32)).cuda(), NG)
    r = {"reversed": np.arange(E)[::-1], "random": bsgen.permutation(3, E),
         "constant": np.zeros(E, dtype=np.int64)}[ranks]
    bs.bs_gs_order_elements(plan, (N + 1) ** 3, torch.from_numpy(np.ascontiguousarray(r).astype(np.int32)).cuda(), 3)
    rs, ci = mesh.csr_inverse(ids, NG)
    for variant in (0, 8):
        with_variant(ctx, variant)
        xL = dev_uniform(NL, 11)
        xG = torch.full((NG,), 7.0, dtype=torch.float64, device="cuda")
        bs.bs_gather(ctx, plan, xL, xG)
        assert np.array_equal(bits(to_host(xG)), bits(ops.gather(rs, ci, to_host(xL))))
    # the derived order copes with masked corners too
    bs.bs_gs_order_elements(plan, (N + 1) ** 3)
    with_variant(ctx, 0)
    xL = dev_uniform(NL, 12)
    xG = torch.empty(NG, dtype=torch.float64, device="cuda")
    bs.bs_gather(ctx, plan, xL, xG)
    assert np.array_equal(bits(to_host(xG)), bits(ops.gather(rs, ci, to_host(xL))))


def test_gather_element_order_errors(ctx):
    K, N = 3, 2
    E, NL, NG = mesh.sizes(K, N)
    d_map, _ = device_map(K, N, 1)
    plan = bs.bs_gs_create(ctx, d_map, NG)
    with pytest.raises(bs.BSError):
        bs.bs_gs_order_elements(plan, 0)
    with pytest.raises(bs.BSError):
        bs.bs_gs_order_elements(plan, 26)  # not a divisor of n_local
    with pytest.raises(bs.BSError):
        bs.bs_gs_order_elements(plan, 9)  # divides n_local but is not (N+1)^3: no order can be derived
    with pytest.raises(ValueError):
        bs.bs_gs_order_elements(plan, 27, torch.zeros(E + 1, dtype=torch.int32, device="cuda"))
    with pytest.raises(bs.BSError):
        bs.bs_gs_order_elements(plan, 27, None, 0)


@pytest.mark.parametrize("K,N,seed,given,group", [(4, 7, 3, False, 1), (5, 4, 7, True, 5), (3, 15, 4, False, 2),
                                                  (6, 2, 2, True, 1), (6, 2, 2, False, 16)])
def test_scatter_tiles_in_element_order(ctx, K, N, seed, given, group):
    # the scatter visits its tiles in the element order too; same bits
    E, NL, NG = mesh.sizes(K, N)
    d_map, ids = device_map(K, N, seed)
    plan = bs.bs_gs_create(ctx, d_map, NG)
    r = torch.from_numpy(bsgen.permutation(seed + 1, E).astype(np.int32)).cuda() if given else None
    bs.bs_gs_order_elements(plan, (N + 1) ** 3, r, group)
    xG_h = host_uniform(NG, 12)
    xL_h = host_uniform(NL, 11)
    ref = ops.scatter(ids, xG_h, xL_h)
    for variant in (0, 1, 2, 8):
        for tpw in (1, 2, 4):
            bs.bs_ctx_set_tune(ctx, "scatter", tpw, 1 << 30, variant)
            xL = torch.from_numpy(xL_h.copy()).cuda()
            bs.bs_gs_scatter(ctx, plan, torch.from_numpy(xG_h).cuda(), xL)
            assert np.array_equal(bits(to_host(xL)), bits(ref)), (variant, tpw)
