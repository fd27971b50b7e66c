"""Pins of the oracle's Gauss-Lobatto rule and derivative matrix (Sec. 3.1)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from conftest import read_golden
from oracle import gl


def _eval(expr):
    return float(eval(expr, {"__builtins__": {}}, {"sqrt": math.sqrt}))


@pytest.mark.parametrize("row", read_golden("gauss_lobatto.txt"), ids=lambda r: "d" + r[0])
def test_closed_form_nodes_weights(row):
    d = int(row[0])
    nodes = [_eval(e) for e in row[1].split(",")]
    weights = [_eval(e) for e in row[2].split(",")]
    x, w = gl.gauss_lobatto(d)
    np.testing.assert_allclose(x, nodes, rtol=0, atol=2e-15)
    np.testing.assert_allclose(w, weights, rtol=0, atol=2e-15)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6])
def test_rule_exact_to_degree_2d_minus_1(d):
    x, w = gl.gauss_lobatto(d)
    for p in range(0, 2 * d):
        exact = float(Fraction(2, p + 1)) if p % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** p) - exact) < 1e-14
    # and not exact one degree higher (the rule has exactly degree 2d-1)
    p = 2 * d
    assert abs(np.sum(w * x ** p) - 2.0 / (p + 1)) > 1e-8


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_derivative_matrix_exact_on_polynomials(d):
    x, _ = gl.gauss_lobatto(d)
    dm = gl.lagrange_derivative_matrix(x)
    for p in range(0, d + 1):
        vals = x ** p
        deriv = p * x ** (p - 1) if p > 0 else np.zeros_like(x)
        np.testing.assert_allclose(dm @ vals, deriv, atol=1e-13)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_summation_by_parts(d):
    x, w = gl.gauss_lobatto(d)
    dm = gl.lagrange_derivative_matrix(x)
    wm = np.diag(w)
    b = np.zeros((d + 1, d + 1))
    b[0, 0], b[d, d] = -1.0, 1.0
    np.testing.assert_allclose(wm @ dm + dm.T @ wm, b, atol=1e-13)


def test_lagrange_interpolation_property():
    x, _ = gl.gauss_lobatto(3)
    np.testing.assert_allclose(gl.lagrange_values(x, x), np.eye(4), atol=1e-14)
