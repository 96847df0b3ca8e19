// Reference-triangle operators (host, FP64), built from their definitions in
// the paper's Section 2: collocation nodes of Warburton's warp-and-blend
// family, an orthonormal hierarchical modal basis with Vandermonde matrix V,
// differentiation D_r = V_r V^{-1}, the mass matrix M = (V V^T)^{-1}, the
// face mass matrix and LIFT = M^{-1} E.
#include "refelem.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace dg {
namespace {

// Orthonormal Jacobi polynomial p_n^(a,b)(x) on [-1,1] (weight
// (1-x)^a (1+x)^b), by the three-term recurrence of orthonormal polynomials.
double jacobi(double x, double a, double b, int n) {
    double g0 = std::pow(2.0, a + b + 1.0) * std::tgamma(a + 1.0) * std::tgamma(b + 1.0) /
                std::tgamma(a + b + 2.0);
    double p0 = 1.0 / std::sqrt(g0);
    if (n == 0) return p0;
    double g1 = (a + 1.0) * (b + 1.0) / (a + b + 3.0) * g0;
    double p1 = ((a + b + 2.0) * x / 2.0 + (a - b) / 2.0) / std::sqrt(g1);
    if (n == 1) return p1;
    auto coef_a = [&](int m) {  // a_m, m >= 1
        double h = 2.0 * m + a + b;
        return 2.0 / h * std::sqrt(m * (m + a + b) * (m + a) * (m + b) / ((h - 1.0) * (h + 1.0)));
    };
    auto coef_b = [&](int m) {  // b_m, m >= 1
        double h = 2.0 * m + a + b;
        return (b * b - a * a) / (h * (h + 2.0));
    };
    double pm1 = p0, pc = p1;
    for (int m = 1; m < n; ++m) {
        double pn = ((x - coef_b(m)) * pc - coef_a(m) * pm1) / coef_a(m + 1);
        pm1 = pc;
        pc = pn;
    }
    return pc;
}

// d/dx p_n^(a,b) = sqrt(n (n+a+b+1)) p_{n-1}^(a+1,b+1).
double jacobi_deriv(double x, double a, double b, int n) {
    if (n == 0) return 0.0;
    return std::sqrt(n * (n + a + b + 1.0)) * jacobi(x, a + 1.0, b + 1.0, n - 1);
}

// Gauss-Lobatto points of order N: -1, 1 and the roots of p_{N-1}^(1,1)
// (proportional to P_N'), found by Newton's method from Chebyshev guesses.
std::vector<double> lobatto(int N) {
    std::vector<double> x(N + 1);
    x[0] = -1.0;
    x[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double z = -std::cos(M_PI * i / N);
        for (int it = 0; it < 100; ++it) {
            double f = jacobi(z, 1.0, 1.0, N - 1);
            double df = jacobi_deriv(z, 1.0, 1.0, N - 1);
            double dz = f / df;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
    }
    std::sort(x.begin(), x.end());
    return x;
}

// Warp of the warp-and-blend construction: interpolant on N+1 equispaced
// points of (Lobatto - equispaced) offsets, divided by 1 - r^2.
double warp(int N, const std::vector<double> &lgl, double r) {
    if (std::fabs(r) >= 1.0 - 1e-10) return 0.0;
    double w = 0.0;
    for (int i = 0; i <= N; ++i) {
        double xi = -1.0 + 2.0 * i / N;
        double li = 1.0;
        for (int m = 0; m <= N; ++m)
            if (m != i) {
                double xm = -1.0 + 2.0 * m / N;
                li *= (r - xm) / (xi - xm);
            }
        w += (lgl[i] - xi) * li;
    }
    return w / (1.0 - r * r);
}

const double kAlpha[9] = {0.0, 0.0, 0.0, 1.4152, 0.1001, 0.2751, 0.9800, 1.0999, 1.2832};

void make_nodes(int P, std::vector<double> &r, std::vector<double> &s) {
    const int Np = n_nodes(P);
    r.assign(Np, 0.0);
    s.assign(Np, 0.0);
    const double alpha = kAlpha[P];
    const std::vector<double> lgl = lobatto(P);
    const double sq3 = std::sqrt(3.0);
    int id = 0;
    for (int n = 0; n <= P; ++n)
        for (int m = 0; m <= P - n; ++m, ++id) {
            double L1 = double(n) / P, L3 = double(m) / P, L2 = 1.0 - L1 - L3;
            double x = -L2 + L3, y = (-L2 - L3 + 2.0 * L1) / sq3;
            double w1 = 4.0 * L2 * L3 * warp(P, lgl, L3 - L2) * (1.0 + (alpha * L1) * (alpha * L1));
            double w2 = 4.0 * L1 * L3 * warp(P, lgl, L1 - L3) * (1.0 + (alpha * L2) * (alpha * L2));
            double w3 = 4.0 * L1 * L2 * warp(P, lgl, L2 - L1) * (1.0 + (alpha * L3) * (alpha * L3));
            x += w1 + std::cos(2.0 * M_PI / 3.0) * w2 + std::cos(4.0 * M_PI / 3.0) * w3;
            y += std::sin(2.0 * M_PI / 3.0) * w2 + std::sin(4.0 * M_PI / 3.0) * w3;
            double l1 = (sq3 * y + 1.0) / 3.0;
            double l2 = (-3.0 * x - sq3 * y + 2.0) / 6.0;
            double l3 = (3.0 * x - sq3 * y + 2.0) / 6.0;
            r[id] = -l2 + l3 - l1;
            s[id] = -l2 - l3 + l1;
        }
}

// Orthonormal mode (i, j) on the triangle and its gradient, through the
// collapsed coordinates a = 2(1+r)/(1-s) - 1, b = s:
// psi = sqrt(2) p_i(a) p_j^(2i+1,0)(b) (1-b)^i.
void mode(double r, double s, int i, int j, double &v, double &dr, double &ds) {
    double b = s;
    double a = (std::fabs(1.0 - s) > 1e-14) ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
    double f = jacobi(a, 0.0, 0.0, i), df = jacobi_deriv(a, 0.0, 0.0, i);
    double g = jacobi(b, 2.0 * i + 1.0, 0.0, j), dg = jacobi_deriv(b, 2.0 * i + 1.0, 0.0, j);
    double om_i = std::pow(1.0 - b, i);
    v = std::sqrt(2.0) * f * g * om_i;
    if (i == 0) {
        dr = 0.0;
        ds = std::sqrt(2.0) * f * dg;
    } else {
        double om = std::pow(1.0 - b, i - 1);
        dr = std::sqrt(2.0) * 2.0 * df * g * om;
        ds = std::sqrt(2.0) * (df * (1.0 + a) * g * om + f * (dg * om_i - i * g * om));
    }
}

// In-place inverse of an n x n row-major matrix (Gauss-Jordan, partial
// pivoting).  Returns false if singular.
bool invert(std::vector<double> &A, int n) {
    std::vector<double> I(n * n, 0.0);
    for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r2 = c + 1; r2 < n; ++r2)
            if (std::fabs(A[r2 * n + c]) > std::fabs(A[piv * n + c])) piv = r2;
        if (std::fabs(A[piv * n + c]) < 1e-300) return false;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(A[c * n + k], A[piv * n + k]);
                std::swap(I[c * n + k], I[piv * n + k]);
            }
        double d = A[c * n + c];
        for (int k = 0; k < n; ++k) {
            A[c * n + k] /= d;
            I[c * n + k] /= d;
        }
        for (int r2 = 0; r2 < n; ++r2)
            if (r2 != c) {
                double f = A[r2 * n + c];
                if (f == 0.0) continue;
                for (int k = 0; k < n; ++k) {
                    A[r2 * n + k] -= f * A[c * n + k];
                    I[r2 * n + k] -= f * I[c * n + k];
                }
            }
    }
    A.swap(I);
    return true;
}

// C = A (m x k) * B (k x n), row-major.
std::vector<double> matmul(const std::vector<double> &A, const std::vector<double> &B, int m, int k,
                           int n) {
    std::vector<double> C(size_t(m) * n, 0.0);
    for (int i = 0; i < m; ++i)
        for (int l = 0; l < k; ++l) {
            double a = A[i * k + l];
            for (int j = 0; j < n; ++j) C[i * n + j] += a * B[l * n + j];
        }
    return C;
}

std::vector<double> transpose(const std::vector<double> &A, int m, int n) {
    std::vector<double> T(size_t(m) * n);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) T[j * m + i] = A[i * n + j];
    return T;
}

// Gauss points of the weight (1-x)^a (1+x)^b on [-1,1] (n points): the
// roots of p_n^(a,b) by Newton's method from Chebyshev guesses, with the
// Christoffel weights 1 / sum_{k<n} p_k(x)^2 of the orthonormal polynomials.
void gauss_jacobi(int n, double a, double b, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            const double f = jacobi(z, a, b, n), df = jacobi_deriv(z, a, b, n);
            const double dz = f / df;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
    }
    std::sort(x.begin(), x.end());
    for (int i = 0; i < n; ++i) {
        double sum = 0.0;
        for (int k = 0; k < n; ++k) {
            const double p = jacobi(x[i], a, b, k);
            sum += p * p;
        }
        w[i] = 1.0 / sum;
    }
}

}  // namespace

double jacobi_orthonormal(double x, double a, double b, int n) { return jacobi(x, a, b, n); }

bool build_weak(int P, WeakOps &w) {
    RefOps o;
    if (!build_reference(P, o)) return false;
    const int Np = o.Np, Nfp = o.Nfp, n = weak_points_per_direction(P);
    w.P = P;
    w.Np = Np;
    w.Nfp = Nfp;
    w.n = n;
    w.ncub = n * n;
    w.ng = n;
    std::vector<double> a, wa, b, wb;
    gauss_jacobi(n, 0.0, 0.0, a, wa);
    gauss_jacobi(n, 1.0, 0.0, b, wb);
    std::vector<int> mi, mj;
    for (int d = 0; d <= P; ++d)
        for (int i = 0; i <= d; ++i) {
            mi.push_back(i);
            mj.push_back(d - i);
        }
    // basis (and derivatives) at points (r, s): modal values times V^{-1}
    auto nodal_at = [&](const std::vector<double> &r, const std::vector<double> &s, std::vector<double> &phi,
                        std::vector<double> &dphr, std::vector<double> &dphs) {
        const int m = int(r.size());
        std::vector<double> Vq(size_t(m) * Np), Vr(size_t(m) * Np), Vs(size_t(m) * Np);
        for (int p = 0; p < m; ++p)
            for (int k = 0; k < Np; ++k) {
                double v, dr, ds;
                mode(r[p], s[p], mi[k], mj[k], v, dr, ds);
                Vq[p * Np + k] = v;
                Vr[p * Np + k] = dr;
                Vs[p * Np + k] = ds;
            }
        phi = matmul(Vq, o.Vinv, m, Np, Np);
        dphr = matmul(Vr, o.Vinv, m, Np, Np);
        dphs = matmul(Vs, o.Vinv, m, Np, Np);
    };
    std::vector<double> rq, sq;
    w.wq.clear();
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            rq.push_back(0.5 * (1.0 + a[i]) * (1.0 - b[j]) - 1.0);
            sq.push_back(b[j]);
            w.wq.push_back(0.5 * wa[i] * wb[j]);
        }
    nodal_at(rq, sq, w.Icub, w.Drc, w.Dsc);
    w.tg = a;
    w.wg = wa;
    // face nodes' 1D Lagrange basis at the Gauss points, through the
    // orthonormal Legendre Vandermonde of the face-node parameters
    std::vector<double> tn(Nfp);
    for (int j = 0; j < Nfp; ++j) tn[j] = o.r[o.fmask[j]];   // face 0: t = r
    std::vector<double> V1(size_t(Nfp) * Nfp), Vg(size_t(n) * Nfp);
    for (int j = 0; j < Nfp; ++j)
        for (int k = 0; k < Nfp; ++k) V1[j * Nfp + k] = jacobi(tn[j], 0.0, 0.0, k);
    for (int g = 0; g < n; ++g)
        for (int k = 0; k < Nfp; ++k) Vg[g * Nfp + k] = jacobi(a[g], 0.0, 0.0, k);
    if (!invert(V1, Nfp)) return false;
    w.If = matmul(Vg, V1, n, Nfp, Nfp);
    w.Drg.clear();
    w.Dsg.clear();
    for (int f = 0; f < 3; ++f) {
        std::vector<double> rg(n), sg(n), phi, dr, ds;
        for (int g = 0; g < n; ++g) {
            const double t = a[g];
            rg[g] = f == 0 ? t : (f == 1 ? -t : -1.0);
            sg[g] = f == 0 ? -1.0 : (f == 1 ? t : -t);
        }
        nodal_at(rg, sg, phi, dr, ds);
        w.Drg.insert(w.Drg.end(), dr.begin(), dr.end());
        w.Dsg.insert(w.Dsg.end(), ds.begin(), ds.end());
    }
    w.Minv = matmul(o.V, transpose(o.V, Np, Np), Np, Np, Np);
    return true;
}

bool build_reference(int P, RefOps &o) {
    if (P < 1 || P > 5) return false;
    const int Np = n_nodes(P), Nfp = P + 1;
    o.P = P;
    o.Np = Np;
    o.Nfp = Nfp;
    make_nodes(P, o.r, o.s);

    // faces in counter-clockwise traversal
    std::vector<int> f0, f1, f2;
    for (int i = 0; i < Np; ++i) {
        if (std::fabs(o.s[i] + 1.0) < 1e-10) f0.push_back(i);
        if (std::fabs(o.r[i] + o.s[i]) < 1e-10) f1.push_back(i);
        if (std::fabs(o.r[i] + 1.0) < 1e-10) f2.push_back(i);
    }
    if ((int)f0.size() != Nfp || (int)f1.size() != Nfp || (int)f2.size() != Nfp) return false;
    std::sort(f0.begin(), f0.end(), [&](int a, int b) { return o.r[a] < o.r[b]; });
    std::sort(f1.begin(), f1.end(), [&](int a, int b) { return o.s[a] < o.s[b]; });
    std::sort(f2.begin(), f2.end(), [&](int a, int b) { return o.s[a] > o.s[b]; });
    o.fmask.clear();
    o.fmask.insert(o.fmask.end(), f0.begin(), f0.end());
    o.fmask.insert(o.fmask.end(), f1.begin(), f1.end());
    o.fmask.insert(o.fmask.end(), f2.begin(), f2.end());

    // modes by total degree, then by i
    std::vector<int> mi, mj;
    for (int d = 0; d <= P; ++d)
        for (int i = 0; i <= d; ++i) {
            mi.push_back(i);
            mj.push_back(d - i);
        }
    o.top_modes.clear();
    for (int n = 0; n < Np; ++n)
        if (mi[n] + mj[n] == P) o.top_modes.push_back(n);

    o.V.assign(Np * Np, 0.0);
    std::vector<double> Vr(Np * Np), Vs(Np * Np);
    for (int p = 0; p < Np; ++p)
        for (int n = 0; n < Np; ++n) {
            double v, dr, ds;
            mode(o.r[p], o.s[p], mi[n], mj[n], v, dr, ds);
            o.V[p * Np + n] = v;
            Vr[p * Np + n] = dr;
            Vs[p * Np + n] = ds;
        }
    o.Vinv = o.V;
    if (!invert(o.Vinv, Np)) return false;
    o.Dr = matmul(Vr, o.Vinv, Np, Np, Np);
    o.Ds = matmul(Vs, o.Vinv, Np, Np, Np);
    std::vector<double> VVt = matmul(o.V, transpose(o.V, Np, Np), Np, Np, Np);
    o.M = VVt;
    if (!invert(o.M, Np)) return false;

    // face mass: 1D orthonormal Legendre Vandermonde at the face nodes'
    // edge parameter (Gauss-Lobatto points), M1 = (V1 V1^T)^{-1}
    std::vector<double> E(size_t(Np) * 3 * Nfp, 0.0);
    for (int f = 0; f < 3; ++f) {
        std::vector<double> V1(Nfp * Nfp);
        for (int i = 0; i < Nfp; ++i) {
            int v = o.fmask[f * Nfp + i];
            double t = (f == 0) ? o.r[v] : (f == 1 ? o.s[v] : -o.s[v]);
            for (int n = 0; n < Nfp; ++n) V1[i * Nfp + n] = jacobi(t, 0.0, 0.0, n);
        }
        std::vector<double> M1 = matmul(V1, transpose(V1, Nfp, Nfp), Nfp, Nfp, Nfp);
        if (!invert(M1, Nfp)) return false;
        for (int i = 0; i < Nfp; ++i)
            for (int j = 0; j < Nfp; ++j)
                E[size_t(o.fmask[f * Nfp + i]) * 3 * Nfp + f * Nfp + j] = M1[i * Nfp + j];
    }
    o.LIFT = matmul(VVt, E, Np, Np, 3 * Nfp);
    return true;
}

}  // namespace dg
