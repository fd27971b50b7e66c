"""One-dimensional Gauss-Lobatto rule and nodal Lagrange derivative matrix.

Oracle (test infrastructure only).  The paper builds its nodal DG basis on
tensor products of the (d+1) one-dimensional Gauss-Lobatto points of ]-1,1[
(Sec. 3.1, eq. map_GL) and on the Lagrange polynomials through those points
(eq. interp_property).  The formulas here are the textbook definitions:

* nodes: -1, +1 and the d-1 roots of P_d' (derivative of the Legendre
  polynomial of degree d);
* weights: w_a = 2 / (d (d+1) P_d(x_a)^2);
* derivative matrix: Dm[a, b] = l_b'(x_a), where l_b is the Lagrange
  polynomial equal to 1 at x_b and 0 at the other nodes.

Pins: closed-form nodes/weights for d = 1..4 (tests/golden/gauss_lobatto.txt),
exactness of the rule up to degree 2d-1, exact differentiation of polynomials
of degree <= d, and the summation-by-parts identity W Dm + Dm^T W = diag(-1,
0, ..., 0, 1).
"""

import numpy as np
from numpy.polynomial import legendre as _leg


def gauss_lobatto(d):
    """Return (nodes, weights) of the (d+1)-point Gauss-Lobatto rule on [-1, 1].

    Nodes are sorted increasingly.  d >= 1.
    """
    if d < 1:
        raise ValueError("degree must be >= 1")
    pd = np.zeros(d + 1)
    pd[d] = 1.0                       # Legendre-series coefficients of P_d
    if d == 1:
        interior = np.array([])
    else:
        interior = np.sort(_leg.legroots(_leg.legder(pd)).real)
    x = np.concatenate(([-1.0], interior, [1.0]))
    w = 2.0 / (d * (d + 1) * _leg.legval(x, pd) ** 2)
    return x, w


def lagrange_derivative_matrix(x):
    """Dm[a, b] = l_b'(x_a) for the Lagrange basis through the points x.

    Written from the product definition l_b(t) = prod_{k != b} (t - x_k) /
    (x_b - x_k), whose derivative is the sum over k != b of the product with
    the k-th factor differentiated.
    """
    n = len(x)
    dm = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            total = 0.0
            for k in range(n):
                if k == b:
                    continue
                prod = 1.0 / (x[b] - x[k])
                for l in range(n):
                    if l == b or l == k:
                        continue
                    prod *= (x[a] - x[l]) / (x[b] - x[l])
                total += prod
            dm[a, b] = total
    return dm


def lagrange_values(x, t):
    """V[p, b] = l_b(t_p): the Lagrange basis through x evaluated at points t."""
    t = np.atleast_1d(np.asarray(t, dtype=float))
    n = len(x)
    v = np.ones((len(t), n))
    for b in range(n):
        for k in range(n):
            if k != b:
                v[:, b] *= (t - x[k]) / (x[b] - x[k])
    return v
