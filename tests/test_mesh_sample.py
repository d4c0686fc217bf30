"""The sampled-mesh helper agrees with the full oracle on small meshes."""

import numpy as np
import pytest

import bsgen
from mesh_sample import MeshSample, seeded_mesh
from oracle import mesh, ops


@pytest.mark.parametrize("K,N,seed", [(4, 3, 1), (5, 1, 2), (3, 7, 3), (6, 2, 4)])
def test_sample_matches_full_oracle(K, N, seed):
    perm, orient = seeded_mesh(K, N, seed)
    E, NL, NG = mesh.sizes(K, N)
    ms = MeshSample(K, N, perm, orient, n_slots=7, seed=seed)
    full = mesh.hex_map(K, N, perm, orient)
    rs, ci = mesh.csr_inverse(full, NG)
    xL = bsgen.uniform(seed, 11, NL)
    g_full = ops.gather(rs, ci, xL)
    got = ms.gather_rows(lambda idx: xL[idx])
    assert np.array_equal(got.view(np.uint64), g_full[ms.g].view(np.uint64))
    assert np.array_equal(ms.degrees(), np.diff(rs)[ms.g])
    l, g = ms.sampled_locals()
    assert np.array_equal(full[l], g)
