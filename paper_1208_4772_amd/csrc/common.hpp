// Device-side helpers shared by the kernels: compile-time node tables,
// packed connectivity, pointwise gas dynamics, numerical flux and boundary
// states.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace dg {

constexpr int kFields = 4;  // rho, rho u, rho v, E

template <int P>
struct Order {
    static constexpr int Np = (P + 1) * (P + 2) / 2;
    static constexpr int Nfp = P + 1;
    static constexpr int Nface = 3 * Nfp;
    static constexpr int EW = 64 / Np;   // elements per wavefront
    static constexpr int EB = 4 * EW;    // elements per 256-thread block
};

// Node id of face node j of face f.  Nodes are numbered in rows of constant
// s (row n has P+1-n nodes), so face 0 is row 0, face 1 the last node of
// each row (increasing s) and face 2 the first node of each row, taken from
// the top row down (counter-clockwise).
__host__ __device__ constexpr int row_start(int P, int n) { return n * (P + 1) - n * (n - 1) / 2; }

__host__ __device__ constexpr int face_node(int P, int f, int j) {
    return f == 0 ? j : (f == 1 ? row_start(P, j) + P - j : row_start(P, P - j));
}

template <int P>
struct FaceTable {
    int v[3 * (P + 1)];
    constexpr FaceTable() : v() {
        for (int f = 0; f < 3; ++f)
            for (int j = 0; j < P + 1; ++j) v[f * (P + 1) + j] = face_node(P, f, j);
    }
};

// Face entries q = f * (P+1) + j that land on each node: up to two (the
// three corners lie on two faces), packed as (q0 + 1) | (q1 + 1) << 8 with 0
// for "none".
template <int P>
struct NodeFaceTable {
    int v[(P + 1) * (P + 2) / 2];
    constexpr NodeFaceTable() : v() {
        for (int q = 0; q < 3 * (P + 1); ++q) {
            const int n = face_node(P, q / (P + 1), q % (P + 1));
            v[n] = v[n] == 0 ? q + 1 : (v[n] | (q + 1) << 8);
        }
    }
};

// Packed face information of an element: 4 bits per face, low 2 bits the
// neighbour's face id, high 2 bits the boundary code.
__host__ __device__ inline int face_nbr_face(int info, int f) { return (info >> (4 * f)) & 3; }
__host__ __device__ inline int face_bc(int info, int f) { return (info >> (4 * f + 2)) & 3; }

enum { BC_INTERIOR = 0, BC_WALL = 1, BC_FARFIELD = 2 };

// Reciprocal and square root: exact (IEEE) in FP64; the single-instruction
// hardware versions (about 1 ulp) in FP32, whose results are checked against
// the FP64 oracle to the FP32 tolerance.
__device__ inline double rcp(double x) { return 1.0 / x; }
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double fsqrt(double x) { return sqrt(x); }
__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double fpow(double x, double y) { return pow(x, y); }
__device__ inline float fpow(float x, float y) { return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x)); }

// p = (gamma-1)(E - (m_x^2 + m_y^2)/(2 rho)), given ir = 1/rho
template <typename T>
__device__ inline T pressure_ir(T g, const T u[kFields], T ir) {
    return (g - T(1)) * (u[3] - T(0.5) * (u[1] * u[1] + u[2] * u[2]) * ir);
}

template <typename T>
__device__ inline T pressure(T g, const T u[kFields]) {
    return pressure_ir(g, u, rcp(u[0]));
}

// Far-field state in primitive form, prepared once on the host.
template <typename T>
struct FarField {
    T q[kFields];     // conserved (rho, rho u, rho v, E)
    T rho, u, v, c;   // primitives and sound speed
    T s;              // entropy p / rho^gamma
    T inv_gm1;        // 1 / (gamma - 1)
};

template <typename T>
FarField<T> make_farfield(double g, const double q[kFields]) {
    const double rho = q[0], u = q[1] / rho, v = q[2] / rho;
    const double p = (g - 1.0) * (q[3] - 0.5 * rho * (u * u + v * v));
    FarField<T> f;
    for (int c = 0; c < kFields; ++c) f.q[c] = T(q[c]);
    f.rho = T(rho);
    f.u = T(u);
    f.v = T(v);
    f.c = T(std::sqrt(g * p / rho));
    f.s = T(p / std::pow(rho, g));
    f.inv_gm1 = T(1.0 / (g - 1.0));
    return f;
}

// Normal flux n.F(u) and the wave speed |v.n| + c.
template <typename T>
__device__ inline void normal_flux(T g, const T u[kFields], T nx, T ny, T fn[kFields], T &lam) {
    T ir = rcp(u[0]);
    T vx = u[1] * ir, vy = u[2] * ir;
    T p = pressure_ir(g, u, ir);
    T vn = vx * nx + vy * ny;
    fn[0] = u[0] * vn;
    fn[1] = u[1] * vn + p * nx;
    fn[2] = u[2] * vn + p * ny;
    fn[3] = (u[3] + p) * vn;
    lam = fabs(vn) + fsqrt(g * p * ir);
}

// Boundary ghost state: slip-wall mirror or characteristic far field.
template <typename T>
__device__ inline void ghost_state(T g, int code, const T um[kFields], T nx, T ny,
                                   const FarField<T> &ff, T up[kFields]) {
    if (code == BC_WALL) {
        T mn = um[1] * nx + um[2] * ny;
        up[0] = um[0];
        up[1] = um[1] - T(2) * mn * nx;
        up[2] = um[2] - T(2) * mn * ny;
        up[3] = um[3];
        return;
    }
    T rhoi = um[0], iri = rcp(rhoi), ui = um[1] * iri, vi = um[2] * iri;
    T pi = pressure_ir(g, um, iri), ci = fsqrt(g * pi * iri);
    T vni = ui * nx + vi * ny;
    T vno = ff.u * nx + ff.v * ny;
    if (vni <= -ci) {
        for (int c = 0; c < kFields; ++c) up[c] = ff.q[c];
        return;
    }
    if (vni >= ci) {
        for (int c = 0; c < kFields; ++c) up[c] = um[c];
        return;
    }
    T gm1 = g - T(1);
    T Rout = vni + T(2) * ci * ff.inv_gm1;
    T Rin = vno - T(2) * ff.c * ff.inv_gm1;
    T vnb = T(0.5) * (Rout + Rin);
    T cb = T(0.25) * gm1 * (Rout - Rin);
    T sb, utb, vtb;
    if (vnb > T(0)) {
        sb = pi * rcp(fpow(rhoi, g));
        utb = ui - vni * nx;
        vtb = vi - vni * ny;
    } else {
        sb = ff.s;
        utb = ff.u - vno * nx;
        vtb = ff.v - vno * ny;
    }
    T rhob = fpow(cb * cb * rcp(g * sb), ff.inv_gm1);
    T pb = rhob * cb * cb * rcp(g);
    T ub = utb + vnb * nx, vb = vtb + vnb * ny;
    up[0] = rhob;
    up[1] = rhob * ub;
    up[2] = rhob * vb;
    up[3] = pb * ff.inv_gm1 + T(0.5) * rhob * (ub * ub + vb * vb);
}

// n.F(u-) - F*(u-, u+) for the local Lax-Friedrichs flux
// F* = (n.F(u-) + n.F(u+))/2 - lam (u+ - u-)/2, lam = max of the two local
// wave speeds:  n.F(u-) - F* = (n.F(u-) - n.F(u+))/2 + lam (u+ - u-)/2.
template <typename T>
__device__ inline void lf_jump(T g, const T um[kFields], const T up[kFields], T nx, T ny,
                               T d[kFields]) {
    T fm[kFields], fp[kFields], lm, lp;
    normal_flux(g, um, nx, ny, fm, lm);
    normal_flux(g, up, nx, ny, fp, lp);
    T lam = lm > lp ? lm : lp;
    for (int c = 0; c < kFields; ++c) {
        T fstar = T(0.5) * (fm[c] + fp[c]) - T(0.5) * lam * (up[c] - um[c]);
        d[c] = fm[c] - fstar;
    }
}

// HLLC state of side K behind its wave of speed SK, contact speed Ss:
// rho_K (S_K - v_n)/(S_K - S*) (1, v + (S* - v_n) n,
// E/rho + (S* - v_n)(S* + p / (rho (S_K - v_n)))).
template <typename T>
__device__ inline void hllc_star(const T u[kFields], T ir, T p, T vn, T nx, T ny, T SK, T Ss,
                                 T out[kFields]) {
    const T f = u[0] * (SK - vn) * rcp(SK - Ss);
    const T dv = Ss - vn;
    out[0] = f;
    out[1] = f * (u[1] * ir + dv * nx);
    out[2] = f * (u[2] * ir + dv * ny);
    out[3] = f * (u[3] * ir + dv * (Ss + p * rcp(u[0] * (SK - vn))));
}

// n.F(u-) - F*(u-, u+) for the HLLC flux (Toro, Spruce and Speares), the
// selectable alternative to local Lax-Friedrichs: Davis wave speeds
// S_L = min(v_n- - c-, v_n+ - c+), S_R = max(v_n- + c-, v_n+ + c+), contact
// speed S* from the two momentum balances; F* = n.F(u-) (S_L >= 0),
// n.F(u-) + S_L (U*_L - u-) (S_L < 0 <= S*), n.F(u+) + S_R (U*_R - u+)
// (S* < 0 < S_R), n.F(u+) (S_R <= 0).
template <typename T>
__device__ inline void hllc_jump(T g, const T um[kFields], const T up[kFields], T nx, T ny, T d[kFields]) {
    T fm[kFields], fp[kFields], lm, lp;
    normal_flux(g, um, nx, ny, fm, lm);
    normal_flux(g, up, nx, ny, fp, lp);
    const T irl = rcp(um[0]), irr = rcp(up[0]);
    const T vnl = (um[1] * nx + um[2] * ny) * irl, vnr = (up[1] * nx + up[2] * ny) * irr;
    const T pl = pressure_ir(g, um, irl), pr = pressure_ir(g, up, irr);
    const T cl = fsqrt(g * pl * irl), cr = fsqrt(g * pr * irr);
    const T SL = fmin(vnl - cl, vnr - cr), SR = fmax(vnl + cl, vnr + cr);
    const T Ss = (pr - pl + um[0] * vnl * (SL - vnl) - up[0] * vnr * (SR - vnr)) *
                 rcp(um[0] * (SL - vnl) - up[0] * (SR - vnr));
    T us[kFields];
    if (SL >= T(0)) {
        for (int c = 0; c < kFields; ++c) d[c] = T(0);
    } else if (Ss >= T(0)) {
        hllc_star(um, irl, pl, vnl, nx, ny, SL, Ss, us);
        for (int c = 0; c < kFields; ++c) d[c] = -SL * (us[c] - um[c]);
    } else if (SR > T(0)) {
        hllc_star(up, irr, pr, vnr, nx, ny, SR, Ss, us);
        for (int c = 0; c < kFields; ++c) d[c] = fm[c] - (fp[c] + SR * (us[c] - up[c]));
    } else {
        for (int c = 0; c < kFields; ++c) d[c] = fm[c] - fp[c];
    }
}

// Numerical-flux difference of the handle's choice: 0 local Lax-Friedrichs,
// 1 HLLC.
enum { RIEMANN_LF = 0, RIEMANN_HLLC = 1 };
template <typename T>
__device__ inline void flux_jump(int riemann, T g, const T um[kFields], const T up[kFields], T nx, T ny,
                                 T d[kFields]) {
    if (riemann == RIEMANN_HLLC)
        hllc_jump(g, um, up, nx, ny, d);
    else
        lf_jump(g, um, up, nx, ny, d);
}

// Time-step bound of one face node (the paper's dt = O(p^-2) with the
// viscous term; reading R11), always in FP64 whatever the state precision:
// 1/2 (P+1)^2 Fscale (|v| + c) + 1/4 (P+1)^4 Fscale^2 eps.
__device__ inline double cfl_bound(double g, const double u[kFields], double fs, double e, double P1) {
    const double ir = 1.0 / u[0];
    const double vx = u[1] * ir, vy = u[2] * ir;
    const double lam = sqrt(vx * vx + vy * vy) + sqrt(g * pressure_ir(g, u, ir) * ir);
    return 0.5 * P1 * P1 * fs * lam + 0.25 * P1 * P1 * P1 * P1 * fs * fs * e;
}

// The same bound for a node that also takes the state check (one division).
__device__ inline double cfl_bound_checked(double g, const double u[kFields], double fs, double e, double P1,
                                           int &bad) {
    const double ir = 1.0 / u[0];
    const double vx = u[1] * ir, vy = u[2] * ir;
    const double p = pressure_ir(g, u, ir);
    if (!(u[0] > 0.0) || !(p > 0.0) || !isfinite(u[1]) || !isfinite(u[2]) || !isfinite(u[3]) || !isfinite(p))
        bad = 1;
    const double lam = sqrt(vx * vx + vy * vy) + sqrt(g * p * ir);
    return 0.5 * P1 * P1 * fs * lam + 0.25 * P1 * P1 * P1 * P1 * fs * fs * e;
}

// State check of one node in FP64: non-finite values, rho <= 0 or p <= 0.
__device__ inline bool bad_state(double g, const double u[kFields]) {
    const double p = pressure(g, u);
    return !(u[0] > 0.0) || !(p > 0.0) || !isfinite(u[1]) || !isfinite(u[2]) || !isfinite(u[3]) ||
           !isfinite(p);
}

// Viscous face-flux difference (sigma Q)*.n - (sigma Q)-.n at a slip wall.
// gm[c] = n.(sigma- Q-) of field c.  The ghost gradient is the mirror image
// implied by the mirror ghost state: mirroring flips a field's normal
// derivative, so rho and E (mirrored unchanged) get (sigma Q)*.n = 0, and
// the momentum (mirrored to m - 2 (m.n) n) keeps only the normal component
// of its normal derivative, (sigma Q)*.n = (gm_m . n) n.
template <typename T>
__device__ inline void wall_visc_jump(const T gm[kFields], T nx, T ny, T d[kFields]) {
    const T gn = gm[1] * nx + gm[2] * ny;
    d[0] = -gm[0];
    d[1] = gn * nx - gm[1];
    d[2] = gn * ny - gm[2];
    d[3] = -gm[3];
}

// Carpenter-Kennedy 2N-storage (5,4) coefficients.
__host__ __device__ inline double rk_a(int s) {
    switch (s) {
        case 1: return -567301805773.0 / 1357537059087.0;
        case 2: return -2404267990393.0 / 2016746695238.0;
        case 3: return -3550918686646.0 / 2091501179385.0;
        case 4: return -1275806237668.0 / 842570457699.0;
        default: return 0.0;
    }
}
__host__ __device__ inline double rk_b(int s) {
    switch (s) {
        case 0: return 1432997174477.0 / 9575080441755.0;
        case 1: return 5161836677717.0 / 13612068292357.0;
        case 2: return 1720146321549.0 / 2090206949498.0;
        case 3: return 3134564353537.0 / 4481467310338.0;
        default: return 2277821191437.0 / 14882151754819.0;
    }
}

}  // namespace dg
