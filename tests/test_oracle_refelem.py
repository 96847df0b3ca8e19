"""Pins of the oracle's reference-triangle operators against brute force,
closed forms and independent constructions (no GPU)."""
from fractions import Fraction
from math import comb, factorial, sqrt

import numpy as np
import pytest
from scipy import special

from oracle.refelem import RefElem, mode_list, ref

PS = [1, 2, 3, 4, 5]

# Gauss-Lobatto points in closed form (roots of (1-x^2) P_N'(x)).
LGL = {
    1: [-1.0, 1.0],
    2: [-1.0, 0.0, 1.0],
    3: [-1.0, -1 / sqrt(5), 1 / sqrt(5), 1.0],
    4: [-1.0, -sqrt(3 / 7), 0.0, sqrt(3 / 7), 1.0],
    5: [-1.0, -sqrt(1 / 3 + 2 * sqrt(7) / 21), -sqrt(1 / 3 - 2 * sqrt(7) / 21),
        sqrt(1 / 3 - 2 * sqrt(7) / 21), sqrt(1 / 3 + 2 * sqrt(7) / 21), 1.0],
}


def monomials(P):
    return [(a, b) for a in range(P + 1) for b in range(P + 1 - a)]


def mono_int_exact(a, b):
    """Exact integral of r^a s^b over T = {r,s >= -1, r+s <= 0} (Fraction).

    r = 2 xi - 1, s = 2 eta - 1 over the unit simplex, and
    int xi^m eta^n = m! n! / (m+n+2)!."""
    tot = Fraction(0)
    for m in range(a + 1):
        for n in range(b + 1):
            c = comb(a, m) * comb(b, n) * 2 ** (m + n) * (-1) ** (a - m + b - n)
            tot += Fraction(c * factorial(m) * factorial(n), factorial(m + n + 2))
    return 4 * tot


def collapsed_rule(n):
    """Tensor rule on T through the collapse r = (1+a)(1-b)/2 - 1, s = b:
    Gauss-Legendre in a, Gauss-Jacobi(1,0) in b."""
    xa, wa = special.roots_legendre(n)
    xb, wb = special.roots_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(xa, xb, indexing="ij")
    W = np.outer(wa, wb) * 0.5
    r = 0.5 * (1 + A) * (1 - B) - 1
    return r.ravel(), B.ravel(), W.ravel()


@pytest.mark.parametrize("P", PS)
def test_edge_nodes_are_gauss_lobatto(P):
    R = ref(P)
    t = R.face_parameters()
    for f in range(3):
        np.testing.assert_allclose(t[f], LGL[P], atol=1e-14)
    # node coordinates of face 0 are (t, -1); face 1 lies on r + s = 0
    np.testing.assert_allclose(R.s[R.Fmask[0]], -1.0, atol=1e-15)
    np.testing.assert_allclose(R.r[R.Fmask[1]] + R.s[R.Fmask[1]], 0.0, atol=1e-14)
    np.testing.assert_allclose(R.r[R.Fmask[2]], -1.0, atol=1e-15)


@pytest.mark.parametrize("P", PS)
def test_nodes_symmetric_under_r_s_swap(P):
    R = ref(P)
    a = np.array(sorted(zip(np.round(R.r, 12), np.round(R.s, 12))))
    b = np.array(sorted(zip(np.round(R.s, 12), np.round(R.r, 12))))
    np.testing.assert_allclose(a, b, atol=1e-12)
    assert len(R.r) == (P + 1) * (P + 2) // 2


def test_node_order_p2():
    R = ref(2)
    expect = [(-1, -1), (0, -1), (1, -1), (-1, 0), (0, 0), (-1, 1)]
    np.testing.assert_allclose(np.stack([R.r, R.s], 1), expect, atol=1e-15)


@pytest.mark.parametrize("P", PS)
def test_basis_orthonormal_by_collapsed_quadrature(P):
    r, s, w = collapsed_rule(P + 3)
    R = ref(P)
    from oracle.refelem import vandermonde
    Vq = vandermonde(P, r, s)
    G = Vq.T @ (w[:, None] * Vq)
    np.testing.assert_allclose(G, np.eye(R.Np), atol=1e-13)


@pytest.mark.parametrize("P", PS)
def test_differentiation_exact_on_polynomials(P):
    R = ref(P)
    r, s = R.r, R.s
    for a, b in monomials(P):
        f = r ** a * s ** b
        dfr = a * r ** max(a - 1, 0) * s ** b
        dfs = b * r ** a * s ** max(b - 1, 0)
        np.testing.assert_allclose(R.Dr @ f, dfr, atol=1e-12)
        np.testing.assert_allclose(R.Ds @ f, dfs, atol=1e-12)
    np.testing.assert_allclose(R.Dr @ np.ones(R.Np), 0, atol=1e-13)


@pytest.mark.parametrize("P", PS)
def test_differentiation_matches_monomial_construction(P):
    R = ref(P)
    r, s = R.r, R.s
    mons = monomials(P)
    Vm = np.stack([r ** a * s ** b for a, b in mons], 1)
    Vmr = np.stack([a * r ** max(a - 1, 0) * s ** b for a, b in mons], 1)
    Vms = np.stack([b * r ** a * s ** max(b - 1, 0) for a, b in mons], 1)
    np.testing.assert_allclose(R.Dr, Vmr @ np.linalg.inv(Vm), atol=1e-11)
    np.testing.assert_allclose(R.Ds, Vms @ np.linalg.inv(Vm), atol=1e-11)


@pytest.mark.parametrize("P", PS)
def test_mass_matrix_brute_force(P):
    """M_ij = int l_i l_j with the Lagrange basis built from monomials and
    integrated exactly."""
    R = ref(P)
    mons = monomials(P)
    Vm = np.stack([R.r ** a * R.s ** b for a, b in mons], 1)
    Cc = np.linalg.inv(Vm)  # l_i = sum_k Cc[k, i] mono_k
    Mmono = np.array([[float(mono_int_exact(a1 + a2, b1 + b2)) for (a2, b2) in mons]
                      for (a1, b1) in mons])
    Mb = Cc.T @ Mmono @ Cc
    np.testing.assert_allclose(R.M, Mb, atol=1e-13)
    assert abs(R.M.sum() - 2.0) < 1e-13       # area of T


@pytest.mark.parametrize("P", PS)
def test_lift_and_face_mass(P):
    R = ref(P)
    np.testing.assert_allclose(R.M @ R.LIFT, R.Emat, atol=1e-13)
    # row sums of the edge mass = Gauss-Lobatto weights 2/(N(N+1) P_N(x)^2)
    x = np.array(LGL[P])
    wl = 2.0 / (P * (P + 1) * special.eval_legendre(P, x) ** 2)
    for f in range(3):
        blk = R.Emat[:, f * R.Nfp:(f + 1) * R.Nfp]
        np.testing.assert_allclose(blk[R.Fmask[f]].sum(1), wl, atol=1e-14)
    # LIFT maps a constant face flux on face 0 to the polynomial whose weak
    # form is the edge integral: int_T l_i (LIFT g) = int_edge l_i g
    g = np.zeros(3 * R.Nfp)
    g[:R.Nfp] = 1.0
    np.testing.assert_allclose((R.M @ (R.LIFT @ g)).sum(), 2.0, atol=1e-13)


@pytest.mark.parametrize("P", PS)
def test_top_modes_are_degree_p(P):
    R = ref(P)
    modes = mode_list(P)
    assert [modes[n][0] + modes[n][1] for n in R.top_modes] == [P] * (P + 1)
    assert list(R.top_modes) == list(range(R.Np - P - 1, R.Np))


def test_invalid_order():
    with pytest.raises(ValueError):
        RefElem(0)
