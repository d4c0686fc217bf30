"""The seven Benchmark-Streaming operations (paper, Table 1), binary64.

Each function is the plain definition of what its operation computes.
Floating-point conventions (the paper fixes binary64 but not the rounding
sequence; these readings are listed with the others in the design notes):

* AXPY and the two vector updates of the fused CG update round each
  product and the sum separately (no fused multiply-add).
* Norm, inner product and the fused update's r.r are returned as the
  correctly rounded value of the exact sum of their terms.  Norm terms are
  fl(x_i*x_i) (times the weight, rounded, when weights are given); inner
  product terms are the exact products x_i*y_i.
* Gather adds the local copies of each global node one at a time, in
  ascending local index, starting from +0.0 (BS6 listing, Section 5).
* Scatter leaves masked (negative-id) local entries untouched (BS7 listing,
  Section 5).

TEST INFRASTRUCTURE ONLY: not part of the library path.
"""

import math

import numpy as np

_SPLIT = 134217729.0  # 2**27 + 1, Veltkamp splitting constant for binary64


def copy(x):
    """BS1 (Table 1, Listing 1): y = x."""
    return np.array(x, dtype=np.float64, copy=True)


def axpy(alpha, x, beta, y):
    """BS2 (Table 1, Listing 2): y <- alpha*x + beta*y.

    Two rounded products and one rounded sum per entry; numpy evaluates each
    operator separately and never contracts to a fused multiply-add.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    ax = np.float64(alpha) * x
    by = np.float64(beta) * y
    return ax + by


def exact_sum(terms):
    """Correctly rounded sum of binary64 terms (Shewchuk/Neumaier, math.fsum)."""
    return math.fsum(np.asarray(terms, dtype=np.float64).ravel().tolist())


def norm_terms(x, w=None):
    """Terms of BS3: fl(x_i*x_i), or fl(w_i*fl(x_i*x_i)) with weights."""
    x = np.asarray(x, dtype=np.float64)
    sq = x * x
    if w is None:
        return sq
    return np.asarray(w, dtype=np.float64) * sq


def norm(x, w=None):
    """BS3 (Table 1, Section 3): alpha = x.x, squared, no square root.

    With weights w (the scattered-form inner product of Section 2, where w is
    one over the node degree) the terms are w_i*x_i^2.  Returned as the
    correctly rounded exact sum of the rounded terms.
    """
    return exact_sum(norm_terms(x, w))


def two_product(a, b):
    """Dekker's exact product: a*b = p + e exactly (no FMA needed).

    Veltkamp splitting of each factor into 26-bit halves; exact for binary64
    inputs whose products neither overflow nor underflow.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    p = a * b
    ca = _SPLIT * a
    ah = ca - (ca - a)
    al = a - ah
    cb = _SPLIT * b
    bh = cb - (cb - b)
    bl = b - bh
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def dot(x, y):
    """BS4 (Table 1): alpha = x.y, the correctly rounded exact inner product."""
    p, e = two_product(x, y)
    return math.fsum(np.concatenate([p, e]).tolist())


def cg_update(alpha, x, p, r, Ap, w=None):
    """BS5 (Table 1; steps 8-10 of Algorithm 1 fused, Section 3).

    x <- x + alpha*p;  r <- r - alpha*Ap;  rho = r.r over the stored new r
    (weighted by w when given).  Returns (x_new, r_new, rho).  The ratio
    beta = rho_new/rho_old of step 10 is a scalar division left to the caller.
    """
    a = np.float64(alpha)
    x_new = np.asarray(x, dtype=np.float64) + a * np.asarray(p, dtype=np.float64)
    r_new = np.asarray(r, dtype=np.float64) - a * np.asarray(Ap, dtype=np.float64)
    return x_new, r_new, norm(r_new, w)


def gather(row_starts, col_ids, xL):
    """BS6 (Table 1, Listing 4): x_G = Z^T x_L.

    Row g of the CSR form of Z^T lists, in ascending order, the local indices
    l with map[l] == g.  Each row is summed one term at a time from +0.0 in
    that order.  Vectorised over rows by degree slot: slot j adds the j-th
    copy of every row that has more than j copies.
    """
    row_starts = np.asarray(row_starts, dtype=np.int64)
    col_ids = np.asarray(col_ids, dtype=np.int64)
    xL = np.asarray(xL, dtype=np.float64)
    n_global = row_starts.size - 1
    deg = np.diff(row_starts)
    acc = np.zeros(n_global, dtype=np.float64)
    for j in range(int(deg.max()) if n_global else 0):
        rows = np.nonzero(deg > j)[0]
        acc[rows] = acc[rows] + xL[col_ids[row_starts[rows] + j]]
    return acc


def scatter(scatter_ids, xG, xL_old):
    """BS7 (Table 1, Listing 5): x_L = Z x_G on unmasked entries.

    Entries whose id is negative are masked out and keep their old value.
    """
    ids = np.asarray(scatter_ids, dtype=np.int64)
    out = np.array(xL_old, dtype=np.float64, copy=True)
    keep = ids >= 0
    out[keep] = np.asarray(xG, dtype=np.float64)[ids[keep]]
    return out
