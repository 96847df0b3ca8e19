"""Pins of the oracle's p-refinement prolongation (no GPU): exact on
polynomials of degree <= P, not on degree P+1, conserves the totals of a
straight mesh exactly, and composes (P -> Q -> R equals P -> R)."""
import numpy as np
import pytest

import meshgen
from oracle import oracle as orc
from oracle.refelem import prolongation, ref


def poly(r, s, coef):
    return sum(c * r ** a * s ** b for (a, b), c in coef.items())


@pytest.mark.parametrize("P,Q", [(1, 2), (2, 3), (2, 5), (3, 4), (4, 5)])
def test_prolongation_is_exact_on_degree_p(P, Q):
    rng = np.random.default_rng(P * 10 + Q)
    coef = {(a, b): rng.normal() for a in range(P + 1) for b in range(P + 1 - a)}
    rp, sp = ref(P).r, ref(P).s
    rq, sq = ref(Q).r, ref(Q).s
    np.testing.assert_allclose(prolongation(P, Q) @ poly(rp, sp, coef), poly(rq, sq, coef), atol=1e-12)
    top = {(P + 1, 0): 1.0}
    assert np.abs(prolongation(P, Q) @ poly(rp, sp, top) - poly(rq, sq, top)).max() > 1e-3


def test_prolongation_composes_and_keeps_identity():
    np.testing.assert_allclose(prolongation(3, 3), np.eye(10), atol=1e-13)
    np.testing.assert_allclose(prolongation(3, 5) @ prolongation(2, 3), prolongation(2, 5), atol=1e-13)


@pytest.mark.parametrize("P,Q", [(2, 3), (2, 4), (3, 5)])
def test_prolongation_conserves_totals_on_straight_mesh(P, Q):
    m = meshgen.periodic_square(5, perm_seed=3)
    Rp, Rq = ref(P), ref(Q)
    xp, yp = meshgen.node_coordinates(m, Rp.r, Rp.s)
    xq, yq = meshgen.node_coordinates(m, Rq.r, Rq.s)
    U = meshgen.isentropic_vortex(xp, yp)
    op = orc.Oracle(m, P, xp, yp)
    oq = orc.Oracle(m, Q, xq, yq)
    np.testing.assert_allclose(oq.totals(orc.prolong(U, P, Q)), op.totals(U), rtol=1e-13, atol=1e-13)
