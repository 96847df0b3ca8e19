"""Pins of the oracle's Persson-Peraire sensor and LDG artificial viscosity
(no GPU)."""
import math

import numpy as np
import pytest
from scipy import special

import meshgen
from oracle import oracle as orc
from oracle.refelem import ref, vandermonde


def one_element_mesh():
    """A 2-element periodic-free patch is not needed: the sensor is local, so
    any mesh works; use a small straight periodic square."""
    return meshgen.periodic_square(3, perm_seed=None, jitter=0.0)


def sensor_oracle(P, eps0=0.3, kappa=1.0, s0=None):
    m = one_element_mesh()
    R = ref(P)
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    return orc.Oracle(m, P, x, y, av=True, av_eps0=eps0, av_kappa=kappa, av_s0=s0), R, m


def state_with_density(R, K, rho_nodal):
    U = np.zeros((K, 4, R.Np))
    U[:, 0, :] = rho_nodal
    U[:, 3, :] = 2.5
    return U


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5])
def test_constant_density_gives_zero_viscosity(P):
    o, R, m = sensor_oracle(P)
    U = state_with_density(R, m.K, np.full(R.Np, 1.3))
    np.testing.assert_array_equal(o.sensor(U), 0.0)


@pytest.mark.parametrize("P", [2, 3, 4, 5])
def test_sensor_ramp_closed_form(P):
    """rho = a psi_0 + d psi_top (orthonormal modes) has S = d^2/(a^2+d^2).
    Choosing d so that log10 S hits s0 - kappa, s0, s0 + kappa and beyond
    gives eps = 0, eps_max/2, eps_max, eps_max with eps_max = eps0 h / P."""
    kappa = 1.0
    s0 = -4.0 * math.log10(P)
    o, R, m = sensor_oracle(P, kappa=kappa)
    h = 2.0 / o.geo["Fscale"].max(1)
    emax = 0.3 * h / P
    a = 1.0
    top = R.top_modes[0]
    for s_target, frac in [(s0 - kappa - 0.3, 0.0), (s0, 0.5), (s0 + kappa + 0.2, 1.0),
                           (s0 + 0.5 * kappa, 0.5 * (1 + math.sin(math.pi / 4)))]:
        S = 10.0 ** s_target
        d = a * math.sqrt(S / (1.0 - S))
        coef = np.zeros(R.Np)
        coef[0] = a
        coef[top] = d
        U = state_with_density(R, m.K, R.V @ coef)
        eps = o.sensor(U)
        np.testing.assert_allclose(eps, frac * emax, rtol=1e-10, atol=1e-300)


def collapsed_rule(n):
    xa, wa = special.roots_legendre(n)
    xb, wb = special.roots_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(xa, xb, indexing="ij")
    return (0.5 * (1 + A) * (1 - B) - 1).ravel(), B.ravel(), (np.outer(wa, wb) * 0.5).ravel()


@pytest.mark.parametrize("P", [2, 3, 4, 5])
def test_sensor_equals_brute_force_projection(P):
    """S_k = ||u - Pi_{P-1} u||^2 / ||u||^2 with Pi the L2 projection onto
    polynomials of degree P-1, computed by least squares in a monomial basis
    under an exact quadrature rule (no modal basis involved)."""
    o, R, m = sensor_oracle(P, kappa=100.0, s0=0.0, eps0=1.0)
    rng = np.random.default_rng(P)
    rho = 1.0 + 0.2 * rng.standard_normal(R.Np)
    U = state_with_density(R, m.K, rho)
    eps = o.sensor(U)[0]
    h = 2.0 / o.geo["Fscale"][0].max()
    emax = h / P
    # invert the (monotone) ramp: eps = emax/2 (1 + sin(pi s / 200))
    s_k = math.asin(2 * eps / emax - 1.0) * 200.0 / math.pi
    # brute force
    rq, sq, wq = collapsed_rule(P + 2)
    mons_full = [(a, b) for a in range(P + 1) for b in range(P + 1 - a)]
    Vm = np.stack([R.r ** a * R.s ** b for a, b in mons_full], 1)
    cu = np.linalg.solve(Vm, rho)
    uq = np.stack([rq ** a * sq ** b for a, b in mons_full], 1) @ cu
    low = [(a, b) for a in range(P) for b in range(P - a)]
    Bq = np.stack([rq ** a * sq ** b for a, b in low], 1)
    W = np.diag(wq)
    c = np.linalg.solve(Bq.T @ W @ Bq, Bq.T @ W @ uq)
    err = uq - Bq @ c
    S = (wq @ err ** 2) / (wq @ uq ** 2)
    assert abs(s_k - math.log10(S)) < 1e-8


@pytest.mark.slow
@pytest.mark.parametrize("P", [1, 2, 3])
def test_viscous_term_solves_heat_equation(P):
    """Inviscid flux off, eps constant: every field obeys u_t = eps Lap u.
    sin(2 pi x/L) sin(2 pi y/L) decays as exp(-2 eps (2 pi/L)^2 t); the error
    must fall at order >= P."""
    L, epsv, T = 10.0, 0.5, 0.25
    R = ref(P)
    errs = []
    for N in (4, 8, 16):
        m = meshgen.periodic_square(N, L, 0.1, 3, 4)
        x, y = meshgen.node_coordinates(m, R.r, R.s)
        o = orc.Oracle(m, P, x, y, no_euler_flux=True, eps_override=epsv, cfl=0.5)
        w = np.sin(2 * np.pi * x / L) * np.sin(2 * np.pi * y / L)
        U0 = np.zeros((m.K, 4, R.Np))
        U0[:, 0] = 2.0 + w
        U0[:, 3] = 5.0 + w
        dt, _ = o.dt(U0)
        n = int(np.ceil(T / dt))
        U, info = o.run(U0, n, dt=T / n)
        decay = math.exp(-2 * epsv * (2 * np.pi / L) ** 2 * info["t"])
        e = np.abs(U[:, 0] - (2.0 + w * decay)).max()
        errs.append(e)
        # mean is conserved exactly by the diffusion operator
        assert abs(o.totals(U)[0] - o.totals(U0)[0]) < 1e-12 * abs(o.totals(U0)[0])
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert (np.diff(errs) < 0).all()
    assert rates[-1] >= P - 0.2, rates


def test_av_rhs_reduces_to_euler_without_viscosity():
    """av on but eps = 0 everywhere (smooth flow below the ramp): the rhs is
    the inviscid one."""
    m = meshgen.periodic_square(6)
    R = ref(3)
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    U = meshgen.isentropic_vortex(x, y, beta=0.5)
    o1 = orc.Oracle(m, 3, x, y, av=False)
    o2 = orc.Oracle(m, 3, x, y, av=True, av_s0=10.0, av_kappa=1.0)
    assert np.abs(o2.sensor(U)).max() == 0.0
    np.testing.assert_allclose(o2.rhs(U), o1.rhs(U), rtol=0, atol=1e-14)


def test_av_is_active_at_a_jump():
    """A density jump inside elements triggers the sensor; the viscous rhs
    then differs from the inviscid one."""
    m = meshgen.periodic_square(6)
    R = ref(3)
    x, y = meshgen.node_coordinates(m, R.r, R.s)
    rho = np.where(x < 5.0, 1.0, 0.5)
    U = np.stack([rho, 0 * rho, 0 * rho, 2.5 + 0 * rho], 1)
    o = orc.Oracle(m, 3, x, y, av=True)
    eps = o.sensor(U)
    assert (eps > 0).sum() > 0 and (eps == 0).sum() > 0
    o0 = orc.Oracle(m, 3, x, y, av=False)
    assert np.abs(o.rhs(U) - o0.rhs(U)).max() > 1e-6
