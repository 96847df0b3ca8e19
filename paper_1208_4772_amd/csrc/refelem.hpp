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

inline int n_nodes(int P) { return (P + 1) * (P + 2) / 2; }

}  // namespace dg
