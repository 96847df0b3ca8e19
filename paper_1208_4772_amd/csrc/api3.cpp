// C ABI of the 3D solver (include/dg3.h): the reference tetrahedron's
// operators (FP64, host), mesh validation, the face node map, device tables
// and the step sequence (bound and dt, then five stages).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dg3.h"
#include "common.hpp"
#include "launch.hpp"
#include "refelem.hpp"

using namespace dg;

namespace {

#define HIP3(expr)                                                                       \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return report_error(DG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

int n3(int P) { return (P + 1) * (P + 2) * (P + 3) / 6; }
int nf3(int P) { return (P + 1) * (P + 2) / 2; }

// Face vertices (indices into the element's 4) and, per face, the two
// volume lattice coordinates that parameterise it.
const int kFaceV[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};

struct Lattice {
    std::vector<int> i, j, k;
};

Lattice lattice3(int P) {
    Lattice L;
    for (int c = 0; c <= P; ++c)
        for (int b = 0; b <= P - c; ++b)
            for (int a = 0; a <= P - c - b; ++a) {
                L.i.push_back(a);
                L.j.push_back(b);
                L.k.push_back(c);
            }
    return L;
}

// Gauss-Jordan inverse with partial pivoting (n x n, row-major); false if
// singular.
bool invert(std::vector<double> A, int n, std::vector<double> &inv) {
    inv.assign(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) inv[size_t(i) * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[size_t(r) * n + c]) > std::fabs(A[size_t(p) * n + c])) p = r;
        if (A[size_t(p) * n + c] == 0.0) return false;
        if (p != c)
            for (int q = 0; q < n; ++q) {
                std::swap(A[size_t(p) * n + q], A[size_t(c) * n + q]);
                std::swap(inv[size_t(p) * n + q], inv[size_t(c) * n + q]);
            }
        const double d = 1.0 / A[size_t(c) * n + c];
        for (int q = 0; q < n; ++q) {
            A[size_t(c) * n + q] *= d;
            inv[size_t(c) * n + q] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = A[size_t(r) * n + c];
            if (f == 0.0) continue;
            for (int q = 0; q < n; ++q) {
                A[size_t(r) * n + q] -= f * A[size_t(c) * n + q];
                inv[size_t(r) * n + q] -= f * inv[size_t(c) * n + q];
            }
        }
    }
    return true;
}

std::vector<double> matmul(const std::vector<double> &A, const std::vector<double> &B, int n, int m, int p) {
    std::vector<double> C(size_t(n) * p, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < m; ++k) {
            const double a = A[size_t(i) * m + k];
            if (a == 0.0) continue;
            for (int j = 0; j < p; ++j) C[size_t(i) * p + j] += a * B[size_t(k) * p + j];
        }
    return C;
}

double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

// Orthonormal modes on the reference tetrahedron through the collapsed
// coordinates a = 2(1+r)/(-s-t) - 1, b = 2(1+s)/(1-t) - 1, c = t:
// 2 sqrt2 p_i(a) p_j^(2i+1,0)(b) (1-b)^i p_k^(2i+2j+2,0)(c) (1-c)^(i+j).
double mode3(double r, double s, double t, int i, int j, int k) {
    const double st = -s - t;
    const double a = std::fabs(st) > 1e-14 ? 2.0 * (1.0 + r) / st - 1.0 : -1.0;
    const double b = std::fabs(1.0 - t) > 1e-14 ? 2.0 * (1.0 + s) / (1.0 - t) - 1.0 : -1.0;
    const double c = t;
    return 2.0 * std::sqrt(2.0) * jacobi_orthonormal(a, 0.0, 0.0, i) *
           jacobi_orthonormal(b, 2.0 * i + 1.0, 0.0, j) * ipow(1.0 - b, i) *
           jacobi_orthonormal(c, 2.0 * (i + j) + 2.0, 0.0, k) * ipow(1.0 - c, i + j);
}

// Orthonormal modes on the triangle (-1,-1), (1,-1), (-1,1):
// sqrt2 p_i(a) p_j^(2i+1,0)(b) (1-b)^i with a = 2(1+r)/(1-s) - 1, b = s.
double mode2(double r, double s, int i, int j) {
    const double a = std::fabs(1.0 - s) > 1e-14 ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
    return std::sqrt(2.0) * jacobi_orthonormal(a, 0.0, 0.0, i) * jacobi_orthonormal(s, 2.0 * i + 1.0, 0.0, j) *
           ipow(1.0 - s, i);
}

// Operators of the reference tetrahedron from their definitions:
// Dr = V_r V^-1 with the monomial basis x^a y^b z^c in x = (1+r)/2, ...
// (d/dr = d/dx / 2); the inverse mass matrix M^-1 = W W^T with W the
// Vandermonde matrix of the orthonormal modes (a nodal basis is W^-T times
// them); face mass matrices of the face Lagrange bases on the reference
// triangle of area 2, (W_f W_f^T)^-1 with the orthonormal triangle modes;
// LIFT = M^-1 E.  fmask: face-major volume node ids.
struct RefOps3 {
    int P = 0, Np = 0, Nfp = 0;
    std::vector<double> r, s, t, Dr, Ds, Dt, LIFT;
    std::vector<int> fmask;
    std::vector<int> bary;   // [4 Nfp][3]: lattice weight of each face vertex at each face node
};

bool build_ref3(int P, RefOps3 &o) {
    const int Np = n3(P), Nfp = nf3(P);
    o.P = P;
    o.Np = Np;
    o.Nfp = Nfp;
    const Lattice L = lattice3(P);
    std::vector<std::tuple<int, int, int>> mons;
    for (int a = 0; a <= P; ++a)
        for (int b = 0; b <= P - a; ++b)
            for (int c = 0; c <= P - a - b; ++c) mons.emplace_back(a, b, c);
    std::vector<double> V(size_t(Np) * Np), Vr(V.size()), Vs(V.size()), Vt(V.size());
    o.r.resize(Np);
    o.s.resize(Np);
    o.t.resize(Np);
    for (int n = 0; n < Np; ++n) {
        const double x = double(L.i[n]) / P, y = double(L.j[n]) / P, z = double(L.k[n]) / P;
        o.r[n] = 2.0 * x - 1.0;
        o.s[n] = 2.0 * y - 1.0;
        o.t[n] = 2.0 * z - 1.0;
        for (int m = 0; m < Np; ++m) {
            const int a = std::get<0>(mons[m]), b = std::get<1>(mons[m]), c = std::get<2>(mons[m]);
            const double xa = ipow(x, a), yb = ipow(y, b), zc = ipow(z, c);
            V[size_t(n) * Np + m] = xa * yb * zc;
            Vr[size_t(n) * Np + m] = a ? 0.5 * a * ipow(x, a - 1) * yb * zc : 0.0;
            Vs[size_t(n) * Np + m] = b ? 0.5 * b * xa * ipow(y, b - 1) * zc : 0.0;
            Vt[size_t(n) * Np + m] = c ? 0.5 * c * xa * yb * ipow(z, c - 1) : 0.0;
        }
    }
    std::vector<double> Vi;
    if (!invert(V, Np, Vi)) return false;
    o.Dr = matmul(Vr, Vi, Np, Np, Np);
    o.Ds = matmul(Vs, Vi, Np, Np, Np);
    o.Dt = matmul(Vt, Vi, Np, Np, Np);
    // the derivative of a constant is zero: each row sums to exactly zero
    // (diagonal = minus the sum of the rest), removing the rounding of the
    // inverse from the derivative of a uniform flux
    for (std::vector<double> *D : {&o.Dr, &o.Ds, &o.Dt})
        for (int i = 0; i < Np; ++i) {
            double off = 0.0;
            for (int j = 0; j < Np; ++j)
                if (j != i) off += (*D)[size_t(i) * Np + j];
            (*D)[size_t(i) * Np + i] = -off;
        }
    // M^-1 = W W^T
    std::vector<double> W(size_t(Np) * Np), Minv(size_t(Np) * Np, 0.0);
    for (int n = 0; n < Np; ++n) {
        int m = 0;
        for (int a = 0; a <= P; ++a)
            for (int b = 0; b <= P - a; ++b)
                for (int c = 0; c <= P - a - b; ++c) W[size_t(n) * Np + m++] = mode3(o.r[n], o.s[n], o.t[n], a, b, c);
    }
    for (int p = 0; p < Np; ++p)
        for (int q = 0; q < Np; ++q) {
            double acc = 0.0;
            for (int m = 0; m < Np; ++m) acc += W[size_t(p) * Np + m] * W[size_t(q) * Np + m];
            Minv[size_t(p) * Np + q] = acc;
        }
    // faces: nodes with k = 0, j = 0, i + j + k = P, i = 0 (increasing node order)
    o.fmask.clear();
    o.bary.clear();
    std::vector<double> E(size_t(Np) * 4 * Nfp, 0.0);
    for (int f = 0; f < 4; ++f) {
        std::vector<int> ids;
        for (int n = 0; n < Np; ++n) {
            const int i = L.i[n], j = L.j[n], k = L.k[n];
            const bool on = f == 0 ? k == 0 : f == 1 ? j == 0 : f == 2 ? (i + j + k == P) : i == 0;
            if (on) ids.push_back(n);
        }
        if (int(ids.size()) != Nfp) return false;
        // face coordinates (u, v) on the unit triangle: (x, y), (x, z),
        // (y, z), (y, z); the area-2 reference triangle is (2u-1, 2v-1)
        std::vector<double> Wf(size_t(Nfp) * Nfp);
        for (int q = 0; q < Nfp; ++q) {
            const int n = ids[q];
            const double x = double(L.i[n]) / P, y = double(L.j[n]) / P, z = double(L.k[n]) / P;
            const double u = f == 0 ? x : f == 1 ? x : y;
            const double v = f == 0 ? y : z;
            int m = 0;
            for (int a = 0; a <= P; ++a)
                for (int b = 0; b <= P - a; ++b) Wf[size_t(q) * Nfp + m++] = mode2(2.0 * u - 1.0, 2.0 * v - 1.0, a, b);
            // lattice weights of the face's three vertices at this node:
            // volume barycentrics (P - i - j - k, i, j, k) of (v1, v2, v3, v4)
            const int lam[4] = {P - L.i[n] - L.j[n] - L.k[n], L.i[n], L.j[n], L.k[n]};
            for (int c = 0; c < 3; ++c) o.bary.push_back(lam[kFaceV[f][c]]);
            o.fmask.push_back(n);
        }
        std::vector<double> WWt(size_t(Nfp) * Nfp, 0.0), Mf;
        for (int p = 0; p < Nfp; ++p)
            for (int q = 0; q < Nfp; ++q) {
                double acc = 0.0;
                for (int m = 0; m < Nfp; ++m) acc += Wf[size_t(p) * Nfp + m] * Wf[size_t(q) * Nfp + m];
                WWt[size_t(p) * Nfp + q] = acc;
            }
        if (!invert(WWt, Nfp, Mf)) return false;
        for (int a = 0; a < Nfp; ++a)
            for (int b = 0; b < Nfp; ++b) E[size_t(ids[a]) * 4 * Nfp + f * Nfp + b] = Mf[size_t(a) * Nfp + b];
    }
    o.LIFT = matmul(Minv, E, Np, Np, 4 * Nfp);
    return true;
}

int check_desc(const dg3_mesh_desc *d) {
    if (!d) return report_error(DG_EINVAL, "desc is NULL");
    if (d->K < 1) return report_error(DG_EINVAL, "K must be >= 1");
    if (d->P < 1 || d->P > 4) return report_error(DG_EINVAL, "P must be in 1..4");
    if (d->precision != DG_FP64_PLAIN && d->precision != DG_FP32)
        return report_error(DG_EINVAL, "precision must be DG_FP64_PLAIN or DG_FP32");
    if (!(d->gamma > 1.0)) return report_error(DG_EINVAL, "gamma must be > 1");
    if (!(d->cfl > 0.0)) return report_error(DG_EINVAL, "cfl must be > 0");
    if (!d->EToV || !d->EToE || !d->EToF || !d->bc || !d->X) return report_error(DG_EINVAL, "null mesh array");
    if (double(d->K) * 5 * n3(d->P) >= 2147483647.0)
        return report_error(DG_EINVAL, "K * 5 * Np must fit in 32 bits");
    return DG_OK;
}

// Validates the connectivity of a desc (ids in range, reciprocal
// neighbours, equal vertex triples on shared faces, self-referencing walls)
// and builds the neighbour node map: a face node is fixed by the lattice
// weights of its face's three global vertices, so the neighbour's node with
// the same weights on the same vertices is its match.  fmap[k][f Nfp + j] =
// kn * 5 * Np + node, or -1 at a wall.
int connect_faces(const dg3_mesh_desc *d, const RefOps3 &o, std::vector<int> &fmap) {
    const int K = d->K, Np = o.Np, Nfp = o.Nfp, NF4 = 4 * Nfp;
    // validation: neighbours in range and reciprocal, walls exactly where
    // the desc says, shared faces with the same vertex triple
    for (long k = 0; k < K; ++k)
        for (int f = 0; f < 4; ++f) {
            const int kn = d->EToE[k * 4 + f], fn = d->EToF[k * 4 + f], code = d->bc[k * 4 + f];
            if (kn < 0 || kn >= K || fn < 0 || fn > 3)
                return report_error(DG_EINVAL, "element " + std::to_string(k) + " face " + std::to_string(f) +
                                                   ": neighbour out of range");
            if (code != DG_BC_INTERIOR && code != DG_BC_WALL)
                return report_error(DG_EINVAL, "bc code must be 0 (interior) or 1 (wall)");
            if (code == DG_BC_WALL) {
                if (kn != k || fn != f)
                    return report_error(DG_EINVAL, "a wall face must point to itself");
                continue;
            }
            if (d->EToE[long(kn) * 4 + fn] != k || d->EToF[long(kn) * 4 + fn] != f)
                return report_error(DG_EINVAL, "element " + std::to_string(k) + " face " + std::to_string(f) +
                                                   ": neighbour not reciprocal");
            int va[3], vb[3];
            for (int c = 0; c < 3; ++c) {
                va[c] = d->EToV[k * 4 + kFaceV[f][c]];
                vb[c] = d->EToV[long(kn) * 4 + kFaceV[fn][c]];
            }
            std::sort(va, va + 3);
            std::sort(vb, vb + 3);
            if (va[0] != vb[0] || va[1] != vb[1] || va[2] != vb[2])
                return report_error(DG_EINVAL, "element " + std::to_string(k) + " face " + std::to_string(f) +
                                                   ": vertex triple differs from the neighbour's");
        }
    // face node map: a face node is fixed by the lattice weights of the
    // face's three (global) vertices; the neighbour's node with the same
    // weights on the same global vertices is the matching node
    fmap.assign(size_t(K) * NF4, -1);
    for (long k = 0; k < K; ++k)
        for (int f = 0; f < 4; ++f) {
            if (d->bc[k * 4 + f] == DG_BC_WALL) {
                for (int j = 0; j < Nfp; ++j) fmap[size_t(k) * NF4 + f * Nfp + j] = -1;
                continue;
            }
            const long kn = d->EToE[k * 4 + f];
            const int fn = d->EToF[k * 4 + f];
            int gv[3], gn[3];
            for (int c = 0; c < 3; ++c) {
                gv[c] = d->EToV[k * 4 + kFaceV[f][c]];
                gn[c] = d->EToV[kn * 4 + kFaceV[fn][c]];
            }
            // position in the neighbour's face of each of this face's vertices
            int perm[3];
            for (int c = 0; c < 3; ++c) {
                perm[c] = -1;
                for (int e = 0; e < 3; ++e)
                    if (gn[e] == gv[c]) perm[c] = e;
                if (perm[c] < 0) return report_error(DG_EINVAL, "internal: face vertices do not match");
            }
            for (int j = 0; j < Nfp; ++j) {
                const int *w = &o.bary[(size_t(f) * Nfp + j) * 3];
                int want[3];
                for (int c = 0; c < 3; ++c) want[perm[c]] = w[c];
                int found = -1;
                for (int jn = 0; jn < Nfp; ++jn) {
                    const int *wn = &o.bary[(size_t(fn) * Nfp + jn) * 3];
                    if (wn[0] == want[0] && wn[1] == want[1] && wn[2] == want[2]) found = jn;
                }
                if (found < 0) return report_error(DG_EINVAL, "internal: face node has no match");
                const int node = o.fmask[size_t(fn) * Nfp + found];
                fmap[size_t(k) * NF4 + f * Nfp + j] = int(kn * 5 * Np + node);
            }
        }
    return DG_OK;
}

// The FP32 stage moves whole tiles as 16-byte vectors.
bool misaligned(const void *p) { return reinterpret_cast<uintptr_t>(p) % 16 != 0; }

}  // namespace

struct dg3_mesh {
    Tet3Mesh m;
    std::vector<void *> allocs;
    hipEvent_t done = nullptr;
    template <typename T>
    int alloc(T **p, size_t count) {
        void *q = nullptr;
        if (hipMalloc(&q, (count ? count : 1) * sizeof(T)) != hipSuccess)
            return report_error(DG_ENOMEM, "device allocation failed");
        allocs.push_back(q);
        *p = static_cast<T *>(q);
        return DG_OK;
    }
    size_t state_bytes() const { return size_t(m.K) * 5 * m.Np * (m.fp32 ? 4 : 8); }
    // offset of each buffer in the work area: the stage kernels move whole
    // tiles as 16-byte vectors, so every buffer starts 256-byte aligned
    size_t slot_bytes() const { return (state_bytes() + 255) / 256 * 256; }
    // two steps captured into a graph on a private stream and replayed on
    // the caller's; rebuilt when the buffers or the fixed step change (the
    // kernels read dt and the bound from device memory)
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    const void *graph_U = nullptr, *graph_work = nullptr;
    double graph_dt = 0.0;
    hipEvent_t t0 = nullptr, t1 = nullptr;   // dg3_run's timing pair, created on first use
    ~dg3_mesh() {
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
        if (graph) (void)hipGraphExecDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (done) (void)hipEventDestroy(done);
        for (void *p : allocs) (void)hipFree(p);
    }
};

namespace {

// One LSERK step: dt from the bound in the slots, then the five stages
// U -> A -> B -> A -> B -> U with the register R, the last of which leaves
// the next step's bound in the slots (a run's first bound: launch_bound3).
hipError_t enqueue_step3(const dg3_mesh *h, void *U, void *work, double dt_fixed, hipStream_t st) {
    const Tet3Mesh &m = h->m;
    char *w = static_cast<char *>(work);
    const size_t sb = h->slot_bytes();
    void *R = w, *A = w + sb, *B = w + 2 * sb;
    void *in[5] = {U, A, B, A, B};
    void *outp[5] = {A, B, A, B, U};
    hipError_t e = launch_dt3(m, dt_fixed, st);
    for (int s = 0; s < 5 && e == hipSuccess; ++s) e = launch_stage3(m, in[s], outp[s], R, nullptr, s, s == 4, st);
    return e;
}

int ensure_graph3(dg3_mesh *h, void *U, void *work, double dt_fixed) {
    if (h->graph && h->graph_U == U && h->graph_work == work && h->graph_dt == dt_fixed) return DG_OK;
    if (h->graph) {
        HIP3(hipGraphExecDestroy(h->graph));
        h->graph = nullptr;
    }
    if (!h->cap_stream) HIP3(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIP3(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed));
    hipError_t e = enqueue_step3(h, U, work, dt_fixed, h->cap_stream);
    if (e == hipSuccess) e = enqueue_step3(h, U, work, dt_fixed, h->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->cap_stream, &g);
    if (e != hipSuccess || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return report_error(DG_EDEVICE, std::string("step capture: ") + hipGetErrorString(e != hipSuccess ? e : ec));
    }
    const hipError_t ei = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return report_error(DG_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    h->graph_U = U;
    h->graph_work = work;
    h->graph_dt = dt_fixed;
    return DG_OK;
}

}  // namespace

extern "C" {

int dg3_reference_nodes(int P, double *r, double *s, double *t) {
    if (P < 1 || P > 4) return report_error(DG_EINVAL, "P must be in 1..4");
    if (!r || !s || !t) return report_error(DG_EINVAL, "null array");
    RefOps3 o;
    if (!build_ref3(P, o)) return report_error(DG_EINVAL, "reference operators: singular matrix");
    std::memcpy(r, o.r.data(), sizeof(double) * o.Np);
    std::memcpy(s, o.s.data(), sizeof(double) * o.Np);
    std::memcpy(t, o.t.data(), sizeof(double) * o.Np);
    return DG_OK;
}

int dg3_reference_operators(int P, double *Dr, double *Ds, double *Dt, double *LIFT, int *fmask) {
    if (P < 1 || P > 4) return report_error(DG_EINVAL, "P must be in 1..4");
    RefOps3 o;
    if (!build_ref3(P, o)) return report_error(DG_EINVAL, "reference operators: singular matrix");
    const size_t nn = size_t(o.Np) * o.Np;
    if (Dr) std::memcpy(Dr, o.Dr.data(), sizeof(double) * nn);
    if (Ds) std::memcpy(Ds, o.Ds.data(), sizeof(double) * nn);
    if (Dt) std::memcpy(Dt, o.Dt.data(), sizeof(double) * nn);
    if (LIFT) std::memcpy(LIFT, o.LIFT.data(), sizeof(double) * o.LIFT.size());
    if (fmask) std::memcpy(fmask, o.fmask.data(), sizeof(int) * o.fmask.size());
    return DG_OK;
}

int dg3_face_map(const dg3_mesh_desc *d, int *fmap) {
    if (int rc = check_desc(d)) return rc;
    if (!fmap) return report_error(DG_EINVAL, "fmap is NULL");
    RefOps3 o;
    if (!build_ref3(d->P, o)) return report_error(DG_EINVAL, "reference operators: singular matrix");
    std::vector<int> m;
    if (int rc = connect_faces(d, o, m)) return rc;
    std::memcpy(fmap, m.data(), sizeof(int) * m.size());
    return DG_OK;
}

int dg3_mesh_setup(const dg3_mesh_desc *d, void *stream, dg3_mesh **out) {
    if (!out) return report_error(DG_EINVAL, "out is NULL");
    *out = nullptr;
    if (int rc = check_desc(d)) return rc;
    const int K = d->K, P = d->P, Np = n3(P), Nfp = nf3(P), NF4 = 4 * Nfp;
    RefOps3 o;
    if (!build_ref3(P, o)) return report_error(DG_EINVAL, "reference operators: singular matrix");
    std::vector<int> fmap;
    if (int rc0 = connect_faces(d, o, fmap)) return rc0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    dg3_mesh *h = new dg3_mesh();
    auto cleanup = [&](int rc) {
        (void)hipStreamSynchronize(st);
        delete h;
        return rc;
    };
#define SETUP3(expr)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return cleanup(report_error(DG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_))); \
    } while (0)
    Tet3Mesh &m = h->m;
    m.K = K;
    m.P = P;
    m.Np = Np;
    m.Nfp = Nfp;
    m.fp32 = d->precision == DG_FP32;
    m.gamma = d->gamma;
    m.cfl = d->cfl;
    int rc;
    double *X_d, *geo64, *scal;
    int *fmap_d, *fmask_d, *count_d, *flag_d;
    unsigned long long *vmax_d;
    if ((rc = h->alloc(&X_d, size_t(K) * 12)) || (rc = h->alloc(&geo64, size_t(K) * 25)) ||
        (rc = h->alloc(&fmap_d, fmap.size())) || (rc = h->alloc(&fmask_d, size_t(NF4))) ||
        (rc = h->alloc(&count_d, 1)) || (rc = h->alloc(&flag_d, 1)) || (rc = h->alloc(&scal, S_NSCAL)) ||
        (rc = h->alloc(&vmax_d, kSlots3)))
        return cleanup(rc);
    SETUP3(hipMemcpyAsync(X_d, d->X, sizeof(double) * size_t(K) * 12, hipMemcpyHostToDevice, st));
    SETUP3(hipMemcpyAsync(fmap_d, fmap.data(), sizeof(int) * fmap.size(), hipMemcpyHostToDevice, st));
    SETUP3(hipMemcpyAsync(fmask_d, o.fmask.data(), sizeof(int) * NF4, hipMemcpyHostToDevice, st));
    SETUP3(hipMemsetAsync(count_d, 0, sizeof(int), st));
    SETUP3(launch_geometry3(K, X_d, geo64, count_d, st));
    int bad = 0;
    SETUP3(hipMemcpyAsync(&bad, count_d, sizeof(int), hipMemcpyDeviceToHost, st));
    SETUP3(hipStreamSynchronize(st));
    if (bad > 0) return cleanup(report_error(DG_EGEOM, std::to_string(bad) + " elements with volume <= 0"));
    m.geo64 = geo64;
    m.fmap = fmap_d;
    m.fmask = fmask_d;
    m.scal = scal;
    m.vmax = vmax_d;
    m.flag = flag_d;
    // the matrix-core A operand in the handle's precision (host copies live
    // until the stream is synchronised below)
    const size_t nA = tet3_mfma_opsA_values(P);
    std::vector<float> opsA32;
    std::vector<double> opsA64;
    if (m.fp32) {
        float *geo32, *opsA_d;
        if ((rc = h->alloc(&geo32, size_t(K) * 25)) || (rc = h->alloc(&opsA_d, nA))) return cleanup(rc);
        SETUP3(launch_cast(geo64, geo32, size_t(K) * 25, st));
        opsA32.resize(nA);
        tet3_mfma_fill_opsA(P, o.Dr.data(), o.Ds.data(), o.Dt.data(), o.LIFT.data(), opsA32.data());
        SETUP3(hipMemcpyAsync(opsA_d, opsA32.data(), sizeof(float) * nA, hipMemcpyHostToDevice, st));
        m.geo32 = geo32;
        m.opsA = opsA_d;
    } else {
        double *opsA_d;
        if ((rc = h->alloc(&opsA_d, nA))) return cleanup(rc);
        opsA64.resize(nA);
        tet3_mfma_fill_opsA64(P, o.Dr.data(), o.Ds.data(), o.Dt.data(), o.LIFT.data(), opsA64.data());
        SETUP3(hipMemcpyAsync(opsA_d, opsA64.data(), sizeof(double) * nA, hipMemcpyHostToDevice, st));
        m.opsA64 = opsA_d;
    }
    SETUP3(launch_reset3(m, st));
    SETUP3(hipEventCreateWithFlags(&h->done, hipEventDisableTiming));
    SETUP3(hipStreamSynchronize(st));
#undef SETUP3
    *out = h;
    return DG_OK;
}

int dg3_mesh_destroy(dg3_mesh *h) {
    if (!h) return report_error(DG_EINVAL, "mesh is NULL");
    if (h->done) (void)hipEventSynchronize(h->done);
    delete h;
    return DG_OK;
}

int dg3_buffer_bytes(const dg3_mesh *h, size_t *state_bytes, size_t *work_bytes) {
    if (!h) return report_error(DG_EINVAL, "mesh is NULL");
    if (state_bytes) *state_bytes = h->state_bytes();
    if (work_bytes) *work_bytes = 3 * h->slot_bytes();
    return DG_OK;
}

int dg3_rhs(dg3_mesh *h, const void *U, void *rhs, void *stream) {
    if (!h || !U || !rhs) return report_error(DG_EINVAL, "null argument");
    if (U == rhs) return report_error(DG_EINVAL, "U and rhs must not alias");
    if (misaligned(U) || misaligned(rhs)) return report_error(DG_EINVAL, "states must be 16-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP3(launch_stage3(h->m, U, nullptr, nullptr, rhs, 0, false, st));
    (void)hipEventRecord(h->done, st);
    return DG_OK;
}

int dg3_run(dg3_mesh *h, void *U, void *work, int nsteps, double dt_fixed, dg_run_stats *stats, void *stream) {
    if (!h || !U || !work) return report_error(DG_EINVAL, "null argument");
    if (nsteps < 0) return report_error(DG_EINVAL, "nsteps must be >= 0");
    if (misaligned(U) || misaligned(work)) return report_error(DG_EINVAL, "U and work must be 16-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Tet3Mesh &m = h->m;
    if (nsteps >= 2)
        if (int rc = ensure_graph3(h, U, work, dt_fixed)) return rc;
    if (!h->t0) HIP3(hipEventCreate(&h->t0));
    if (!h->t1) HIP3(hipEventCreate(&h->t1));
    hipEvent_t e0 = h->t0, e1 = h->t1;
    HIP3(launch_reset3(m, st));
    HIP3(hipEventRecord(e0, st));
    if (nsteps > 0) HIP3(launch_bound3(m, U, st));
    int n = 0;
    if (nsteps >= 2)
        for (; n + 2 <= nsteps; n += 2) HIP3(hipGraphLaunch(h->graph, st));
    for (; n < nsteps; ++n) HIP3(enqueue_step3(h, U, work, dt_fixed, st));
    HIP3(hipEventRecord(e1, st));
    double scal[S_NSCAL];
    int flag = 0;
    HIP3(hipMemcpyAsync(scal, m.scal, sizeof(scal), hipMemcpyDeviceToHost, st));
    HIP3(hipMemcpyAsync(&flag, m.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    (void)hipEventRecord(h->done, st);
    HIP3(hipStreamSynchronize(st));
    float ms = 0.f;
    HIP3(hipEventElapsedTime(&ms, e0, e1));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->steps = nsteps;
        stats->status = flag ? DG_ENONFINITE : DG_OK;
        stats->t = scal[S_T];
        stats->dt_min = nsteps ? scal[S_DTMIN] : 0.0;
        stats->dt_max = scal[S_DTMAX];
        stats->wall_s = ms * 1e-3;
        stats->dof_updates_per_s = ms > 0 ? double(m.K) * 5 * m.Np * 5.0 * nsteps / (ms * 1e-3) : 0.0;
    }
    if (flag) return report_error(DG_ENONFINITE, "state became non-finite or non-positive (rho or p)");
    return DG_OK;
}

}  // extern "C"
