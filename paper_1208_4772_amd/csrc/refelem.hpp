// Reference-triangle operators of the nodal DG method (host, FP64).
#pragma once
#include <vector>

namespace dg {

struct RefOps {
    int P = 0, Np = 0, Nfp = 0;
    std::vector<double> r, s;       // nodes [Np]
    std::vector<int> fmask;         // [3][Nfp], counter-clockwise per face
    std::vector<double> V, Vinv;    // [Np][Np] row-major
    std::vector<double> Dr, Ds;     // [Np][Np]
    std::vector<double> M;          // [Np][Np]
    std::vector<double> LIFT;       // [Np][3*Nfp]
    std::vector<int> top_modes;     // modal ids of total degree P
};

// Builds every operator of order P (1..5).  Returns false on a bad order or
// a singular Vandermonde matrix.
bool build_reference(int P, RefOps &out);

// Operators of the over-integrated weak form of order P: a collapsed
// (conical) product rule of n x n points on the reference triangle, exact
// for total degree 2n - 1 >= 3P (n Gauss-Legendre points in a, n
// Gauss-Jacobi points of weight (1 - b) in b, r = (1+a)(1-b)/2 - 1, s = b,
// weight w_a w_b / 2), and n Gauss-Legendre points on every face.
struct WeakOps {
    int P = 0, Np = 0, Nfp = 0, n = 0, ncub = 0, ng = 0;
    std::vector<double> wq;         // [ncub]
    std::vector<double> Icub;       // [ncub][Np] nodal basis at the cubature points
    std::vector<double> Drc, Dsc;   // [ncub][Np] its derivatives there
    std::vector<double> tg, wg;     // [ng] face Gauss points (CCW face parameter) and weights
    std::vector<double> If;         // [ng][Nfp] face-node Lagrange basis at the Gauss points
    std::vector<double> Drg, Dsg;   // [3][ng][Np] basis derivatives at each face's Gauss points
    std::vector<double> Minv;       // [Np][Np] inverse reference mass matrix V V^T
};
bool build_weak(int P, WeakOps &out);
inline int weak_points_per_direction(int P) { return (3 * P + 2) / 2; }

inline int n_nodes(int P) { return (P + 1) * (P + 2) / 2; }

// Jacobi polynomial p_n^(a,b)(x) of unit norm on [-1,1] under the weight
// (1-x)^a (1+x)^b.
double jacobi_orthonormal(double x, double a, double b, int n);

}  // namespace dg
