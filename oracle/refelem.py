"""Reference-triangle operators for the CPU oracle.

TEST INFRASTRUCTURE ONLY: the oracle is imported by the tests, by the smoke
check and by the benchmark's CPU-baseline leg.  The solver library never
imports, links or calls anything in ``oracle/``.

Everything is FP64 and follows the paper's construction of the local
operators (Section 2, "The discontinuous Galerkin method"), restricted to the
2D reference triangle T = {r, s >= -1, r + s <= 0} with vertices
v1=(-1,-1), v2=(1,-1), v3=(-1,1):

* collocation nodes: warp-and-blend nodes of Warburton (2006), the node family
  the paper cites for its collocation points;
* an orthonormal, hierarchical modal basis psi_j and the Vandermonde matrix
  V_ij = psi_j(r_i)  (f = V f_hat);
* differentiation D_r = V_r V^{-1}, D_s = V_s V^{-1} (paper: D_r = V_r V^{-1}),
  evaluated at the collocation nodes (nodal strong form);
* mass matrix M = (V V^T)^{-1} (the exact L2 mass matrix of the nodal basis,
  which is what the paper's cubature mass matrix integrates);
* face mass: per face, the 1D mass matrix of the face's Lagrange basis, and
  LIFT = M^{-1} E (the paper's M_k^{-1} M_dOmega on the reference element).

Independent pieces deliberately use library routines (SciPy's Jacobi
polynomials and gamma function, NumPy's Legendre roots) rather than
hand-rolled recurrences.
"""
from __future__ import annotations

import functools
import math

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy import special

# Warp-and-blend blending exponents per order (Warburton 2006, the
# Lebesgue-constant-optimised values).
ALPHA_OPT = {1: 0.0, 2: 0.0, 3: 1.4152, 4: 0.1001, 5: 0.2751, 6: 0.9800,
             7: 1.0999, 8: 1.2832}


def n_nodes(P: int) -> int:
    return (P + 1) * (P + 2) // 2


# ---------------------------------------------------------------------------
# 1D ingredients
# ---------------------------------------------------------------------------

def jacobi_normalized(x, alpha, beta, n):
    """Jacobi polynomial P_n^(alpha,beta)(x) scaled to unit norm on [-1,1]
    under the weight (1-x)^alpha (1+x)^beta."""
    x = np.asarray(x, dtype=np.float64)
    h = (2.0 ** (alpha + beta + 1) / (2 * n + alpha + beta + 1)
         * math.exp(special.gammaln(n + alpha + 1) + special.gammaln(n + beta + 1)
                    - special.gammaln(n + alpha + beta + 1) - special.gammaln(n + 1)))
    return special.eval_jacobi(n, alpha, beta, x) / math.sqrt(h)


def jacobi_normalized_deriv(x, alpha, beta, n):
    """d/dx of :func:`jacobi_normalized` (uses dP_n/dx = (n+a+b+1)/2 P_{n-1}^(a+1,b+1))."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.zeros_like(x)
    h = (2.0 ** (alpha + beta + 1) / (2 * n + alpha + beta + 1)
         * math.exp(special.gammaln(n + alpha + 1) + special.gammaln(n + beta + 1)
                    - special.gammaln(n + alpha + beta + 1) - special.gammaln(n + 1)))
    return (0.5 * (n + alpha + beta + 1)
            * special.eval_jacobi(n - 1, alpha + 1, beta + 1, x) / math.sqrt(h))


def gauss_lobatto_points(N: int) -> np.ndarray:
    """The N+1 Legendre-Gauss-Lobatto points on [-1,1]: the end points and the
    roots of P_N'."""
    if N == 1:
        return np.array([-1.0, 1.0])
    inner = npleg.Legendre.basis(N).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


# ---------------------------------------------------------------------------
# nodes
# ---------------------------------------------------------------------------

def _warp(N: int, rout: np.ndarray) -> np.ndarray:
    """Warp of Warburton's construction: the polynomial interpolant (on N+1
    equispaced points of [-1,1]) of the offset from equispaced to
    Gauss-Lobatto points, divided by 1 - r^2 (zero at the ends)."""
    lgl = gauss_lobatto_points(N)
    req = np.linspace(-1.0, 1.0, N + 1)
    w = np.zeros_like(rout)
    for i in range(N + 1):
        li = np.ones_like(rout)
        for m in range(N + 1):
            if m != i:
                li *= (rout - req[m]) / (req[i] - req[m])
        w += (lgl[i] - req[i]) * li
    inner = np.abs(rout) < 1.0 - 1e-10
    out = np.zeros_like(rout)
    out[inner] = w[inner] / (1.0 - rout[inner] ** 2)
    return out


def nodes(P: int, alpha: float | None = None):
    """Warp-and-blend nodes (r, s) on T, ordered in rows of constant s
    (increasing s), increasing r within a row.  ``alpha``: the blending
    exponent (default: the table's value for this order)."""
    alpha = ALPHA_OPT[P] if alpha is None else float(alpha)
    L1, L3 = [], []
    for n in range(P + 1):          # row index: L1 = n/P  (s = 2 L1 - 1)
        for m in range(P + 1 - n):  # position in the row: L3 = m/P
            L1.append(n / P)
            L3.append(m / P)
    L1 = np.array(L1)
    L3 = np.array(L3)
    L2 = 1.0 - L1 - L3
    # equilateral triangle with vertices (-1,-1/sqrt3), (1,-1/sqrt3), (0,2/sqrt3)
    x = -L2 + L3
    y = (-L2 - L3 + 2.0 * L1) / math.sqrt(3.0)
    b1, b2, b3 = 4 * L2 * L3, 4 * L1 * L3, 4 * L1 * L2
    w1 = b1 * _warp(P, L3 - L2) * (1.0 + (alpha * L1) ** 2)
    w2 = b2 * _warp(P, L1 - L3) * (1.0 + (alpha * L2) ** 2)
    w3 = b3 * _warp(P, L2 - L1) * (1.0 + (alpha * L3) ** 2)
    c2, s2 = math.cos(2 * math.pi / 3), math.sin(2 * math.pi / 3)
    c3, s3 = math.cos(4 * math.pi / 3), math.sin(4 * math.pi / 3)
    x = x + w1 + c2 * w2 + c3 * w3
    y = y + s2 * w2 + s3 * w3
    # back to barycentric coordinates, then to (r, s)
    l1 = (math.sqrt(3.0) * y + 1.0) / 3.0
    l2 = (-3.0 * x - math.sqrt(3.0) * y + 2.0) / 6.0
    l3 = (3.0 * x - math.sqrt(3.0) * y + 2.0) / 6.0
    r = -l2 + l3 - l1
    s = -l2 - l3 + l1
    return r, s


def face_masks(P: int, r: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Node ids of the three faces, each in counter-clockwise traversal:
    face 0 v1->v2 (s=-1), face 1 v2->v3 (r+s=0), face 2 v3->v1 (r=-1)."""
    tol = 1e-10
    f0 = np.nonzero(np.abs(s + 1.0) < tol)[0]
    f0 = f0[np.argsort(r[f0])]
    f1 = np.nonzero(np.abs(r + s) < tol)[0]
    f1 = f1[np.argsort(s[f1])]
    f2 = np.nonzero(np.abs(r + 1.0) < tol)[0]
    f2 = f2[np.argsort(-s[f2])]
    fm = np.stack([f0, f1, f2])
    assert fm.shape == (3, P + 1)
    return fm


# ---------------------------------------------------------------------------
# modal basis
# ---------------------------------------------------------------------------

def mode_list(P: int):
    """(i, j) exponents ordered by total degree i + j, then by i."""
    return [(i, d - i) for d in range(P + 1) for i in range(d + 1)]


def _collapse(r, s):
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    a = np.where(np.abs(1.0 - s) > 1e-14, 2.0 * (1.0 + r) / np.where(np.abs(1.0 - s) > 1e-14, 1.0 - s, 1.0) - 1.0, -1.0)
    return a, s


def basis(r, s, i, j):
    """Orthonormal PKDO mode psi_ij = sqrt2 Phat_i(a) Phat_j^(2i+1,0)(b) (1-b)^i."""
    a, b = _collapse(r, s)
    return (math.sqrt(2.0) * jacobi_normalized(a, 0, 0, i)
            * jacobi_normalized(b, 2 * i + 1, 0, j) * (1.0 - b) ** i)


def basis_grad(r, s, i, j):
    """(d psi/dr, d psi/ds) by the chain rule through the collapsed
    coordinates a = 2(1+r)/(1-s) - 1, b = s."""
    a, b = _collapse(r, s)
    f = jacobi_normalized(a, 0, 0, i)
    df = jacobi_normalized_deriv(a, 0, 0, i)
    g = jacobi_normalized(b, 2 * i + 1, 0, j)
    dg = jacobi_normalized_deriv(b, 2 * i + 1, 0, j)
    if i == 0:
        dr = np.zeros_like(a)
        ds = f * dg
    else:
        om = (1.0 - b) ** (i - 1)
        dr = 2.0 * df * g * om
        ds = df * (1.0 + a) * g * om + f * (dg * (1.0 - b) ** i - i * g * om)
    return math.sqrt(2.0) * dr, math.sqrt(2.0) * ds


def vandermonde(P, r, s):
    return np.stack([basis(r, s, i, j) for (i, j) in mode_list(P)], axis=1)


def grad_vandermonde(P, r, s):
    g = [basis_grad(r, s, i, j) for (i, j) in mode_list(P)]
    return np.stack([a for a, _ in g], axis=1), np.stack([b for _, b in g], axis=1)


# ---------------------------------------------------------------------------
# operators
# ---------------------------------------------------------------------------

class RefElem:
    """All reference operators of order P (FP64, row-major numpy arrays)."""

    def __init__(self, P: int):
        if P < 1 or P > 8:
            raise ValueError("1 <= P <= 8")
        self.P = P
        self.Np = n_nodes(P)
        self.Nfp = P + 1
        self.r, self.s = nodes(P)
        self.Fmask = face_masks(P, self.r, self.s)
        self.V = vandermonde(P, self.r, self.s)
        self.Vinv = np.linalg.inv(self.V)
        Vr, Vs = grad_vandermonde(P, self.r, self.s)
        self.Dr = Vr @ self.Vinv
        self.Ds = Vs @ self.Vinv
        self.M = np.linalg.inv(self.V @ self.V.T)
        # face mass: 1D Lagrange basis on the face nodes, orthonormal Legendre
        # Vandermonde in the face parameter t in [-1, 1] (CCW direction)
        E = np.zeros((self.Np, 3 * self.Nfp))
        tpar = self.face_parameters()
        for f in range(3):
            t = tpar[f]
            V1 = np.stack([jacobi_normalized(t, 0, 0, n) for n in range(self.Nfp)], axis=1)
            M1 = np.linalg.inv(V1 @ V1.T)
            for i in range(self.Nfp):
                E[self.Fmask[f, i], f * self.Nfp:(f + 1) * self.Nfp] = M1[i]
        self.Emat = E
        self.LIFT = self.V @ (self.V.T @ E)
        # modes of total degree P (dropped by the smoothness sensor)
        self.top_modes = np.array([n for n, (i, j) in enumerate(mode_list(P)) if i + j == P])

    def face_parameters(self):
        """Edge parameter t in [-1,1] of each face node, in the face's CCW order."""
        r, s = self.r, self.s
        fm = self.Fmask
        return np.stack([r[fm[0]], s[fm[1]], -s[fm[2]]])


@functools.lru_cache(maxsize=None)
def ref(P: int) -> RefElem:
    return RefElem(P)


def prolongation(P: int, Q: int) -> np.ndarray:
    """(Np(Q), Np(P)) matrix evaluating a degree-P nodal polynomial at the
    order-Q nodes (p-refinement, Section 5: the modal coefficients padded with
    zeros).  The modes are ordered by total degree, so the first Np(P) modes
    of order Q are exactly those of degree <= P."""
    if Q < P:
        raise ValueError("Q >= P")
    return ref(Q).V[:, :n_nodes(P)] @ ref(P).Vinv


# ---------------------------------------------------------------------------
# cubature: the paper's over-integrated weak form
# ---------------------------------------------------------------------------

def cubature_points_per_direction(P: int) -> int:
    """n for the rules below: exact for total degree 2n - 1 >= 3P."""
    return (3 * P + 2) // 2


def triangle_cubature(n: int):
    """Collapsed (conical) product rule on T with n x n points (Stroud): n
    Gauss-Legendre points in a and n Gauss-Jacobi points of weight (1 - b)
    in b (the Jacobian of the collapse), mapped by r = (1+a)(1-b)/2 - 1,
    s = b; weights w_a w_b / 2.  Exact for polynomials of total degree
    <= 2n - 1 on T (area 2)."""
    a, wa = special.roots_legendre(n)
    b, wb = special.roots_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(a, b, indexing="ij")
    WA, WB = np.meshgrid(wa, wb, indexing="ij")
    r = 0.5 * (1.0 + A) * (1.0 - B) - 1.0
    return r.ravel(), B.ravel(), (0.5 * WA * WB).ravel()


class WeakOperators:
    """Operators of the over-integrated weak form of order P: the nodal basis
    and its derivatives at the cubature points (Icub, Drc, Dsc), the Gauss
    rule of each face (wg at points tg of the face parameter, the same
    counter-clockwise parameter as the face nodes), the face nodes' 1D
    Lagrange basis at the Gauss points (If) and the basis derivatives at each
    face's Gauss points (Drg, Dsg), for the metric terms there."""

    def __init__(self, P: int):
        R = ref(P)
        self.P = P
        n = cubature_points_per_direction(P)
        self.rq, self.sq, self.wq = triangle_cubature(n)
        self.ncub = self.wq.size
        self.Icub = vandermonde(P, self.rq, self.sq) @ R.Vinv
        Vr, Vs = grad_vandermonde(P, self.rq, self.sq)
        self.Drc, self.Dsc = Vr @ R.Vinv, Vs @ R.Vinv
        self.tg, self.wg = special.roots_legendre(n)
        self.ng = n
        tn = R.face_parameters()[0]                       # the same LGL parameters on every face
        V1n = np.stack([jacobi_normalized(tn, 0, 0, m) for m in range(R.Nfp)], axis=1)
        V1g = np.stack([jacobi_normalized(self.tg, 0, 0, m) for m in range(R.Nfp)], axis=1)
        self.If = V1g @ np.linalg.inv(V1n)
        t = self.tg
        face_rs = [(t, -np.ones_like(t)), (-t, t), (-np.ones_like(t), -t)]
        Drg, Dsg = [], []
        for rg, sg in face_rs:
            a, b = grad_vandermonde(P, rg, sg)
            Drg.append(a @ R.Vinv)
            Dsg.append(b @ R.Vinv)
        self.Drg, self.Dsg = np.stack(Drg), np.stack(Dsg)
        self.face_rs = face_rs


@functools.lru_cache(maxsize=None)
def weak_ops(P: int) -> WeakOperators:
    return WeakOperators(P)

