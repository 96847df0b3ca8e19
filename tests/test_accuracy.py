"""Host-side diagnostics of the accuracy reports, checked against closed
forms (no GPU)."""
import math

import numpy as np
import pytest

import meshgen
from paper_1208_4772_amd import accuracy, dg


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_line_rule_exact_on_polynomials(n):
    # Gauss-Lobatto points with n nodes: weights exact to degree 2n - 3,
    # differentiation exact to degree n - 1
    from numpy.polynomial.legendre import Legendre
    if n == 2:
        t = np.array([-1.0, 1.0])
    else:
        t = np.concatenate([[-1.0], np.sort(Legendre.basis(n - 1).deriv().roots()), [1.0]])
    w, D = accuracy._line_rule(t)
    for d in range(2 * n - 2):
        exact = (1.0 - (-1.0) ** (d + 1)) / (d + 1)
        assert abs(w @ t ** d - exact) < 1e-13, d
    for d in range(n):
        np.testing.assert_allclose(D @ t ** d, d * t ** max(d - 1, 0) if d else 0 * t, atol=1e-12)


def cylinder(P=4, scale=0.05):
    r, s = dg.reference_nodes(P)
    return meshgen.make_case("cylinder", r, s, scale=scale, P=P)


def test_uniform_pressure_gives_no_force():
    case = cylinder()
    geo = accuracy.Geometry(case)
    loads = geo.wall_loads(case.U0, case.freestream)
    assert abs(loads["CL"]) < 1e-12 and abs(loads["CD"]) < 1e-12
    assert abs(loads["cp_min"]) < 1e-12


def test_linear_pressure_gives_buoyancy_of_the_body():
    # p = p0 + c y on the fluid side: the pressure force on the body is
    # -c * (body area) in y, and the curved (quartic) wall encloses the unit
    # circle's area to a few parts in 1e6 on this mesh
    case = cylinder()
    geo = accuracy.Geometry(case)
    q = case.freestream
    p0 = 0.4 * (q[3] - 0.5 * q[1] ** 2 / q[0])
    c = 0.01
    U = case.U0.copy()
    p = p0 + c * case.y
    U[:, 3] = p / 0.4 + 0.5 * (U[:, 1] ** 2 + U[:, 2] ** 2) / U[:, 0]
    loads = geo.wall_loads(U, q)
    qdyn = 0.5 * q[1] ** 2 / q[0]
    assert abs(loads["CL"] * qdyn - (-c * math.pi)) < 1e-5 * c * math.pi
    assert abs(loads["CD"]) < 1e-12


def test_mass_weights_sum_to_the_domain_area():
    r, s = dg.reference_nodes(3)
    case = meshgen.make_case("vortex", r, s, P=3)
    geo = accuracy.Geometry(case)
    assert abs(geo.area - 100.0) < 1e-10
    # totals of a uniform state are the state times the area
    T = geo.totals(meshgen.uniform((case.K, case.Np), case.freestream))
    np.testing.assert_allclose(T, 100.0 * case.freestream, rtol=1e-12)


def test_entropy_error_of_freestream_and_of_a_uniform_offset():
    case = cylinder(P=2)
    geo = accuracy.Geometry(case)
    assert geo.entropy_error(case.U0, case.freestream) < 1e-15
    # scaling the pressure by (1 + d) at fixed density scales s by (1 + d)
    U = case.U0.copy()
    q = case.freestream
    ke = 0.5 * (U[:, 1] ** 2 + U[:, 2] ** 2) / U[:, 0]
    U[:, 3] = (U[:, 3] - ke) * 1.001 + ke
    assert abs(geo.entropy_error(U, q) - 1e-3) < 1e-12


def test_state_errors():
    a = np.ones((3, 4, 6))
    b = a.copy()
    b[1, 2, 3] += 0.5
    e = accuracy.state_errors(b, a)
    assert e["max_abs"] == 0.5
    assert abs(e["rel_l2"] - 0.5 / math.sqrt(a.size)) < 1e-15


def test_shock_position_is_the_last_rise_through_critical_cp():
    """Upper-surface C_p = C_p* + 2 (x - 0.6) with a wiggle through C_p*
    near the leading edge: the shock is the crossing at x = 0.6 (linear
    between nodes, so exact); no crossing gives NaN."""
    r, s = dg.reference_nodes(3)
    case = meshgen.make_case("airfoil", r, s, scale=0.01, P=3)
    geo = accuracy.Geometry(case)
    q = case.freestream
    g = 1.4
    rho0, u0, v0 = q[0], q[1] / q[0], q[2] / q[0]
    p0 = (g - 1) * (q[3] - 0.5 * rho0 * (u0 * u0 + v0 * v0))
    qd = 0.5 * rho0 * (u0 * u0 + v0 * v0)
    cstar = accuracy.critical_cp(0.8)
    x = case.x
    cp = np.where(x < 0.15, cstar + (x - 0.1),
                  np.where(x < 0.2, cstar + 0.05 - 2.0 * (x - 0.15), cstar + 2.0 * (x - 0.6)))
    U = np.stack([np.ones_like(x), 0 * x, 0 * x, (p0 + qd * cp) / (g - 1)], 1)
    assert geo.wall_loads(U, q)["shock_x"] == pytest.approx(0.6, abs=1e-9)
    U[:, 3] = (p0 + qd * (cstar + 0.1)) / (g - 1)
    assert math.isnan(geo.wall_loads(U, q)["shock_x"])
