"""Oracle values for a sample of a large mesh, computed one row at a time.

For meshes too large for the oracle to map in full, the oracle maps only a
sample of element slots plus every slot whose element touches them (a node
of lattice element e is shared only with the elements at offsets -1..1 of e
in each axis).  That yields, for every global node of the sampled slots,
its complete list of local copies, so gather rows and scatter entries can be
computed exactly for the sample.
"""

import numpy as np

import bsgen
from oracle import mesh


class MeshSample:
    def __init__(self, K, N, perm, orient, n_slots, seed=0):
        self.K, self.N = K, N
        self.Np3 = (N + 1) ** 3
        E = K ** 3
        perm = np.asarray(perm, dtype=np.int64)
        orient = np.asarray(orient, dtype=np.int64)
        inv = np.empty(E, dtype=np.int64)
        inv[perm] = np.arange(E)
        rng = np.random.default_rng(seed)
        slots = np.unique(np.concatenate([rng.choice(E, min(n_slots, E), replace=False), [0, E - 1]]))
        e = perm[slots]
        q = np.stack([e % K, (e // K) % K, e // (K * K)], axis=1)
        near = []
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    n = q + np.array([dx, dy, dz])
                    ok = np.all((n >= 0) & (n < K), axis=1)
                    near.append(inv[n[ok, 0] + K * (n[ok, 1] + K * n[ok, 2])])
        self.slots = slots
        self.all_slots = np.unique(np.concatenate([slots] + near))
        rows = mesh.hex_map(K, N, perm[self.all_slots], orient[self.all_slots]).reshape(-1, self.Np3)
        self.rows = {int(s): rows[i] for i, s in enumerate(self.all_slots)}
        # copies of every global node of the sampled slots, ascending local index
        want = np.unique(np.concatenate([self.rows[int(s)] for s in slots]))
        local = (self.all_slots[:, None] * self.Np3 + np.arange(self.Np3)[None, :]).ravel()
        ids = rows.ravel()
        keep = np.isin(ids, want)
        order = np.lexsort((local[keep], ids[keep]))
        self.g = want
        gi, li = ids[keep][order], local[keep][order]
        starts = np.searchsorted(gi, want)
        ends = np.searchsorted(gi, want, side="right")
        self.copies = [li[a:b] for a, b in zip(starts, ends)]

    def sampled_locals(self):
        """Local indices of the sampled slots and their oracle global ids."""
        l = (self.slots[:, None] * self.Np3 + np.arange(self.Np3)[None, :]).ravel()
        g = np.concatenate([self.rows[int(s)] for s in self.slots])
        return l, g

    def gather_rows(self, xL_at):
        """Oracle gather of the sampled rows; xL_at(idx) returns local values."""
        allc = np.concatenate(self.copies)
        vals = dict(zip(allc.tolist(), xL_at(allc).tolist()))
        out = np.empty(len(self.g))
        for i, c in enumerate(self.copies):
            acc = 0.0
            for l in c.tolist():
                acc = acc + vals[l]
            out[i] = acc
        return out

    def degrees(self):
        return np.array([len(c) for c in self.copies])


def seeded_mesh(K, N, seed):
    E = K ** 3
    return bsgen.permutation(seed, E), bsgen.orientations(seed, E)
