"""The library's host box-mesh builder against the oracle's (no GPU needed)."""

import numpy as np
import pytest

from oracle import mesh

import paper_2009_10917_amd as bs  # noqa: E402


@pytest.mark.parametrize("E,N", [(1, 2), (7, 3), (8, 2), (20, 4), (27, 2), (100, 5), (343, 2), (4096, 2)])
def test_box_map_matches_oracle(E, N):
    got, ng = bs.bs_mesh_box_map_host(E, N)
    ids, ng_o = mesh.box_map(E, N)
    assert ng == ng_o and np.array_equal(got.astype(np.int64), ids)


def test_box_map_rejects_bad_sizes():
    with pytest.raises(bs.BSError):
        bs.bs_mesh_box_map_host(0, 3)
    with pytest.raises(bs.BSError):
        bs.bs_mesh_box_map_host(5, 0)
