"""Pins for the Dubiner basis and the quadrature rules (Sec. 2.2, Eq. dubiner).

Checks against facts fixed by mathematics, computed independently with
sympy: the closed-form diagonal mass 2/((2i+1)(i+j+1)), orthogonality,
exact derivatives of the basis written from its definition with sympy's
Jacobi polynomials, and exact monomial integrals over the reference
triangle.
"""
import itertools

import numpy as np
import pytest
import sympy as sp

from oracle import basis

r, s = sp.symbols("r s")


def sym_dubiner(i, j):
    a = 2 * (1 + r) / (1 - s) - 1
    expr = sp.legendre(i, a) * ((1 - s) / 2) ** i * sp.jacobi(j, 2 * i + 1, 0, s)
    return sp.expand(sp.cancel(sp.together(expr)))


def tri_integral(f):
    return sp.integrate(sp.integrate(f, (r, -1, -s)), (s, -1, 1))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mass_closed_form_and_orthogonality(p):
    modes = basis.mode_list(p)
    syms = [sym_dubiner(i, j) for i, j in modes]
    M = sp.Matrix(len(modes), len(modes), lambda a, b: tri_integral(syms[a] * syms[b]))
    closed = [sp.Rational(2, (2 * i + 1) * (i + j + 1)) for i, j in modes]
    for a in range(len(modes)):
        assert M[a, a] == closed[a]
        for b in range(len(modes)):
            if a != b:
                assert M[a, b] == 0
    np.testing.assert_allclose(basis.mass_diag(p), [float(c) for c in closed], rtol=0, atol=1e-15)


def test_p1_explicit_forms():
    # phi_10 = (1 + 2r + s)/2 and phi_01 = (1 + 3s)/2 follow from the definition
    assert sp.simplify(sym_dubiner(1, 0) - (1 + 2 * r + s) / 2) == 0
    assert sp.simplify(sym_dubiner(0, 1) - (1 + 3 * s) / 2) == 0


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_values_and_gradients_match_definition(p):
    rng = np.random.default_rng(1)
    pts = []
    while len(pts) < 12:
        a, b = rng.uniform(-1, 1, 2)
        if a + b <= 0:
            pts.append((a, b))
    pts += [(-1.0, 1.0), (1.0, -1.0), (-1.0, -1.0)]     # includes the collapsed vertex
    rr = np.array([q[0] for q in pts]); ss = np.array([q[1] for q in pts])
    phi, dr, ds = basis.eval_basis(p, rr, ss)
    for m, (i, j) in enumerate(basis.mode_list(p)):
        f = sym_dubiner(i, j)
        fr, fs = sp.diff(f, r), sp.diff(f, s)
        for n, (a, b) in enumerate(pts):
            assert abs(phi[m, n] - float(f.subs({r: a, s: b}))) < 1e-13
            assert abs(dr[m, n] - float(fr.subs({r: a, s: b}))) < 1e-12
            assert abs(ds[m, n] - float(fs.subs({r: a, s: b}))) < 1e-12


@pytest.mark.parametrize("p,degree", [(0, 2), (1, 2), (2, 4), (3, 6)])
def test_area_rule_exact_to_its_degree(p, degree):
    qr, qs, qw = basis.area_rule(p)
    for a, b in itertools.product(range(degree + 1), repeat=2):
        if a + b > degree:
            continue
        exact = float(tri_integral(r ** a * s ** b))
        approx = float(np.sum(qw * qr ** a * qs ** b))
        assert abs(approx - exact) < 1e-14, (a, b)


def test_area_rule_p2_not_exact_beyond_degree_4():
    qr, qs, qw = basis.area_rule(2)
    exact = float(tri_integral(s ** 5))
    assert abs(np.sum(qw * qs ** 5) - exact) > 1e-6


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_edge_rule_exact_degree_2p_plus_1(p):
    t, w = basis.edge_rule(p)
    x = sp.symbols("x")
    for d in range(2 * p + 2):
        exact = float(sp.integrate(x ** d, (x, -1, 1)))
        assert abs(np.sum(w * t ** d) - exact) < 1e-14
    assert np.all(np.diff(t) > 0) and np.allclose(t, -t[::-1], atol=0, rtol=0) or np.allclose(t, -t[::-1], atol=1e-16)


def test_edge_points_and_vertex_inverse():
    T = basis.Tables(1)
    # p=1 vertex values: rows are vertices, columns modes
    np.testing.assert_allclose(T.phi_v, [[1, -1, -1], [1, 1, -1], [1, 0, 2]], atol=1e-15)
    np.testing.assert_allclose(T.V1inv @ T.V1, np.eye(3), atol=1e-15)
    # edge k runs from v_k to v_{k+1}
    for k in range(3):
        a = basis.edge_point(k, -1.0); b = basis.edge_point(k, 1.0)
        np.testing.assert_allclose(a, basis.REF_VERTS[k]); np.testing.assert_allclose(b, basis.REF_VERTS[(k + 1) % 3])
