"""One step of the batched workload on one instance, from the single operations.

Each instance is a box mesh (mesh.box_map) with global vectors x, y, p, r, Ap
(length N_G) and local vectors xL, pL, wL (length N_L).  One step applies
the seven streaming operations of Table 1 once each, then one CG iteration
(Algorithm 1, steps 5-11) with the operator A = Z^T Z, i.e. scatter then
gather, which is diag(degree):

   1  y  = x                          BS1
   2  y  = alpha x + beta y           BS2
   3  norm = sum wL xL^2              BS3
   4  dot  = x . y                    BS4
   5  x += alpha p, r -= alpha Ap,    BS5, rr = r . r
   6  xL = Z x                        BS7
   7  y  = Z^T xL                     BS6
   8  pL = Z p                        BS7
   9  Ap = Z^T pL                     BS6
  10  pAp = p . Ap, a = rr / pAp      BS4
  11  x += a p, r -= a Ap,            BS5, rr2 = r . r
  12  p  = r + (rr2 / rr) p           BS2

alpha and beta of steps 2 and 5 are the same for every instance; a and
b = rr2 / rr are each instance's own.

TEST INFRASTRUCTURE ONLY: not part of the library path.
"""

import numpy as np

from . import mesh, ops

SCALARS = ("norm", "dot", "rr", "pAp", "alpha", "rr2", "beta")


def step(scatter_ids, n_global, v, alpha, beta):
    """Apply one step to the dict of float64 vectors v (copied).

    Returns (vectors, scalars) after the step.
    """
    rs, ci = mesh.csr_inverse(scatter_ids, n_global)
    x, y, p, r, Ap = (np.array(v[k], dtype=np.float64) for k in ("x", "y", "p", "r", "Ap"))
    xL, pL, wL = (np.array(v[k], dtype=np.float64) for k in ("xL", "pL", "wL"))
    out = {}
    y = ops.copy(x)
    y = ops.axpy(alpha, x, beta, y)
    out["norm"] = ops.norm(xL, wL)
    out["dot"] = ops.dot(x, y)
    x, r, out["rr"] = ops.cg_update(alpha, x, p, r, Ap)
    xL = ops.scatter(scatter_ids, x, xL)
    y = ops.gather(rs, ci, xL)
    pL = ops.scatter(scatter_ids, p, pL)
    Ap = ops.gather(rs, ci, pL)
    out["pAp"] = ops.dot(p, Ap)
    out["alpha"] = out["rr"] / out["pAp"]
    x, r, out["rr2"] = ops.cg_update(out["alpha"], x, p, r, Ap)
    out["beta"] = out["rr2"] / out["rr"]
    p = ops.axpy(1.0, r, out["beta"], p)
    return dict(x=x, y=y, p=p, r=r, Ap=Ap, xL=xL, pL=pL, wL=wL), out


def cg_iterations(scatter_ids, n_global, b, tol=1e-12, max_iter=64):
    """CG on A = Z^T Z from x = 0 using steps 8-12 only; returns (x, iterations).

    A is diagonal with at most as many distinct entries as there are distinct
    node degrees, so exact CG ends within that many iterations.
    """
    rs, ci = mesh.csr_inverse(scatter_ids, n_global)
    nl = len(scatter_ids)
    x = np.zeros(n_global)
    r = np.array(b, dtype=np.float64)
    p = r.copy()
    rr = ops.norm(r)
    rr0 = rr
    it = 0
    while it < max_iter and rr > tol * tol * rr0:
        Ap = ops.gather(rs, ci, ops.scatter(scatter_ids, p, np.zeros(nl)))
        a = rr / ops.dot(p, Ap)
        x, r, rr2 = ops.cg_update(a, x, p, r, Ap)
        p = ops.axpy(1.0, r, rr2 / rr, p)
        rr = rr2
        it += 1
    return x, it
