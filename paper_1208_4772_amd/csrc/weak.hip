// The paper's over-integrated weak form (Section 2, eqs. stiffness, mass,
// face_mass, semidiscrete) as a selectable variant of the stage kernel:
//
//   M_k dU/dt = V - S,
//   V_i = sum_q w_q J_q [dphi_i/dr (r_x F + r_y G) + dphi_i/ds (s_x F + s_y G)](x_q)
//   S_i = sum_f sum_g w_g sJ_fg phi_i(x_fg) F*(u-, u+)_fg
//
// with the state interpolated to a cubature rule exact for degree 3P and to
// Gauss points on the faces, the fluxes evaluated there, and the per-element
// mass matrix M_k (J M_ref on a straight element, its inverse precomputed by
// Cholesky factorisation on a curved one).  The paper forms S_x and M_k^{-1}
// per curved element (Section 4); here a curved element keeps its metric
// terms per cubature point and its inverse mass matrix, a straight one five
// numbers.  The contractions run on the VALUs in the handle's precision
// (FP64 or FP32); the setup (metric terms at cubature and face points, mass
// matrices, Cholesky) runs in FP64 on the GPU.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "launch.hpp"

namespace dg {
namespace {

constexpr int kWBlock = 256;

template <int P>
struct WShape {
    static constexpr int Np = (P + 1) * (P + 2) / 2, Nfp = P + 1;
    static constexpr int n = (3 * P + 2) / 2;         // points per direction / per face
    static constexpr int NQ = n * n, NG = n;
};

// Elements per block: LDS of U, the cubature fluxes (2 x 4 x NQ), the face
// fluxes (4 x 3 NG) and the right-hand side vector within a budget per
// precision.  Measured at P = 5 on 1M elements: FP32 runs fastest with small
// blocks (36 KB: 11 elements per block at P = 5, four blocks per CU), FP64
// with large ones (60 KB: its registers, not the LDS, cap the resident
// waves).  The reference operators stay in global memory (caches): staged
// in LDS they cost more resident blocks than the reads they save.
constexpr int kWeakBudgetF32 = 36 * 1024, kWeakBudgetF64 = 60 * 1024;

template <typename T, int P>
constexpr int weak_elems() {
    using S = WShape<P>;
    constexpr int per = (8 * S::Np + 8 * S::NQ + 12 * S::NG) * int(sizeof(T));
    constexpr int e = (sizeof(T) == 4 ? kWeakBudgetF32 : kWeakBudgetF64) / per;
    return e < 1 ? 1 : (e > 32 ? 32 : e);
}

template <typename T>
struct WeakArgs {
    int K, stage, mode, riemann;
    T g, ra, rb;
    FarField<T> ff;
    const T *__restrict__ Uin;
    T *__restrict__ Uout;
    T *__restrict__ R;
    T *__restrict__ rhs;
    const int *__restrict__ nbr;
    const int *__restrict__ finfo;
    const T *__restrict__ ops;     // Icub | Drc | Dsc | wq | If | Minv
    const T *__restrict__ geoA;    // [K][5] r_x s_x r_y s_y J (straight elements)
    const T *__restrict__ geoF;    // [K][3][NG][3] n_x n_y w_g sJ
    const T *__restrict__ geoC;    // [Kc][NQ][4] w_q J (r_x, s_x, r_y, s_y)
    const T *__restrict__ minv;    // [Kc][Np][Np] inverse mass matrix
    const int *__restrict__ widx;  // [K] curved slot or -1
    const double *__restrict__ dt;
};

template <typename T, int P>
__global__ __launch_bounds__(kWBlock) void k_stage_weak(WeakArgs<T> a) {
    using S = WShape<P>;
    constexpr int Np = S::Np, Nfp = S::Nfp, NQ = S::NQ, NG = S::NG, EB = weak_elems<T, P>();
    __shared__ T sU[EB][kFields][Np];
    __shared__ T sA[EB][kFields][NQ];
    __shared__ T sB[EB][kFields][NQ];
    __shared__ T sS[EB][kFields][3 * NG];
    __shared__ T sb[EB][kFields][Np];
    const long k0 = (long)blockIdx.x * EB;
    const int nel = (int)min((long)EB, (long)a.K - k0);
    const int tid = threadIdx.x;

    const T *Icub = a.ops, *Drc = Icub + NQ * Np, *Dsc = Drc + NQ * Np, *wq = Dsc + NQ * Np;
    const T *If = wq + NQ, *Minv = If + NG * Nfp;

    for (int z = tid; z < nel * kFields * Np; z += kWBlock) (&sU[0][0][0])[z] = a.Uin[k0 * kFields * Np + z];
    __syncthreads();

    // volume fluxes at the cubature points, weighted and mapped
    for (int z = tid; z < nel * NQ; z += kWBlock) {
        const int el = z / NQ, q = z - el * NQ;
        const long k = k0 + el;
        T u[kFields] = {};
        for (int j = 0; j < Np; ++j) {
            const T phi = Icub[q * Np + j];
#pragma unroll
            for (int c = 0; c < kFields; ++c) u[c] += phi * sU[el][c][j];
        }
        const T ir = rcp(u[0]);
        const T vx = u[1] * ir, vy = u[2] * ir, p = pressure_ir(a.g, u, ir);
        const T F[kFields] = {u[1], u[1] * vx + p, u[2] * vx, (u[3] + p) * vx};
        const T G[kFields] = {u[2], u[1] * vy, u[2] * vy + p, (u[3] + p) * vy};
        const int cs = a.widx[k];
        T wrx, wsx, wry, wsy;
        if (cs < 0) {
            const T *gk = a.geoA + k * 5;
            const T wJ = wq[q] * gk[4];
            wrx = wJ * gk[0];
            wsx = wJ * gk[1];
            wry = wJ * gk[2];
            wsy = wJ * gk[3];
        } else {
            const T *gq = a.geoC + ((long)cs * NQ + q) * 4;
            wrx = gq[0];
            wsx = gq[1];
            wry = gq[2];
            wsy = gq[3];
        }
#pragma unroll
        for (int c = 0; c < kFields; ++c) {
            sA[el][c][q] = wrx * F[c] + wry * G[c];
            sB[el][c][q] = wsx * F[c] + wsy * G[c];
        }
    }
    // numerical fluxes at the face Gauss points, times w_g sJ
    for (int z = tid; z < nel * 3 * NG; z += kWBlock) {
        const int el = z / (3 * NG), fg = z - el * 3 * NG, f = fg / NG, gq = fg - f * NG;
        const long k = k0 + el;
        T um[kFields] = {}, up[kFields] = {};
        for (int j = 0; j < Nfp; ++j) {
            const T l = If[gq * Nfp + j];
            const int v = face_node(P, f, j);
#pragma unroll
            for (int c = 0; c < kFields; ++c) um[c] += l * sU[el][c][v];
        }
        const T *gf = a.geoF + ((k * 3 + f) * NG + gq) * 3;
        const T nx = gf[0], ny = gf[1], ws = gf[2];
        const int info = a.finfo[k];
        const int code = face_bc(info, f);
        if (code == BC_INTERIOR) {
            // the neighbour's face node Nfp-1-j sits on this face's node j
            const long kn = a.nbr[k * 3 + f];
            const int fn = face_nbr_face(info, f);
            for (int j = 0; j < Nfp; ++j) {
                const T l = If[gq * Nfp + j];
                const int v = face_node(P, fn, Nfp - 1 - j);
#pragma unroll
                for (int c = 0; c < kFields; ++c) up[c] += l * a.Uin[(kn * kFields + c) * Np + v];
            }
        } else {
            ghost_state(a.g, code, um, nx, ny, a.ff, up);
        }
        T fm[kFields], lm, d[kFields];
        normal_flux(a.g, um, nx, ny, fm, lm);
        flux_jump(a.riemann, a.g, um, up, nx, ny, d);
#pragma unroll
        for (int c = 0; c < kFields; ++c) sS[el][c][fg] = ws * (fm[c] - d[c]);
    }
    __syncthreads();
    // V - S per node, the four fields together (each operator entry read
    // once for all of them)
    constexpr NodeFaceTable<P> kNF;
    for (int z = tid; z < nel * Np; z += kWBlock) {
        const int el = z / Np, i = z - el * Np;
        T b[kFields] = {};
        for (int q = 0; q < NQ; ++q) {
            const T dr = Drc[q * Np + i], ds = Dsc[q * Np + i];
#pragma unroll
            for (int c = 0; c < kFields; ++c) b[c] += dr * sA[el][c][q] + ds * sB[el][c][q];
        }
        const int nq = kNF.v[i];
        if (nq) {
            for (int t = 0; t < 2; ++t) {
                const int e = t == 0 ? (nq & 255) - 1 : (nq >> 8) - 1;
                if (e < 0) continue;
                const int f = e / Nfp, j = e - f * Nfp;
                for (int gq = 0; gq < NG; ++gq) {
                    const T l = If[gq * Nfp + j];
#pragma unroll
                    for (int c = 0; c < kFields; ++c) b[c] -= l * sS[el][c][f * NG + gq];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < kFields; ++c) sb[el][c][i] = b[c];
    }
    __syncthreads();
    // M_k^{-1} (V - S), then the Runge-Kutta update, the four fields of a
    // node together
    const T dt = a.mode ? T(*a.dt) : T(0);
    for (int z = tid; z < nel * Np; z += kWBlock) {
        const int el = z / Np, i = z - el * Np;
        const long k = k0 + el;
        const int cs = a.widx[k];
        T val[kFields] = {};
        if (cs < 0) {
            for (int j = 0; j < Np; ++j) {
                const T mij = Minv[i * Np + j];
#pragma unroll
                for (int c = 0; c < kFields; ++c) val[c] += mij * sb[el][c][j];
            }
            const T J = a.geoA[k * 5 + 4];
#pragma unroll
            for (int c = 0; c < kFields; ++c) val[c] = val[c] / J;
        } else {
            const T *mk = a.minv + (long)cs * Np * Np + i * Np;
            for (int j = 0; j < Np; ++j) {
                const T mij = mk[j];
#pragma unroll
                for (int c = 0; c < kFields; ++c) val[c] += mij * sb[el][c][j];
            }
        }
#pragma unroll
        for (int c = 0; c < kFields; ++c) {
            const long idx = k0 * kFields * Np + (el * kFields + c) * Np + i;
            if (a.mode == 0) {
                a.rhs[idx] = val[c];
            } else {
                const T rr = (a.stage == 0) ? dt * val[c] : a.ra * a.R[idx] + dt * val[c];
                a.R[idx] = rr;
                a.Uout[idx] = sU[el][c][i] + a.rb * rr;
            }
        }
    }
}

// ---- setup (FP64) ---------------------------------------------------------

// Per element: metric terms at the first cubature point (all of them for a
// straight element), the unit normal and w_g sJ at every face Gauss point;
// for a curved element the mapped cubature weights per point and the mass
// matrix sum_q w_q J_q phi_i phi_j.  Coordinates relative to the element's
// first node (as the nodal geometry).
template <int P>
__global__ void k_weak_geometry(int K, const double *__restrict__ x, const double *__restrict__ y,
                                const double *__restrict__ ops, const double *__restrict__ Drg,
                                const double *__restrict__ Dsg, const double *__restrict__ wg,
                                const int *__restrict__ widx, double *__restrict__ geoA,
                                double *__restrict__ geoF, double *__restrict__ geoC,
                                double *__restrict__ mass, int *__restrict__ count) {
    using S = WShape<P>;
    constexpr int Np = S::Np, NQ = S::NQ, NG = S::NG;
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const double *Icub = ops, *Drc = Icub + NQ * Np, *Dsc = Drc + NQ * Np, *wq = Dsc + NQ * Np;
    double xl[Np], yl[Np];
    for (int j = 0; j < Np; ++j) {
        xl[j] = x[k * Np + j] - x[k * Np];
        yl[j] = y[k * Np + j] - y[k * Np];
    }
    const int cs = widx[k];
    double *mk = cs >= 0 ? mass + (long)cs * Np * Np : nullptr;
    if (mk)
        for (int z = 0; z < Np * Np; ++z) mk[z] = 0.0;
    for (int q = 0; q < NQ; ++q) {
        double xr = 0, xs = 0, yr = 0, ys = 0;
        for (int j = 0; j < Np; ++j) {
            xr += Drc[q * Np + j] * xl[j];
            xs += Dsc[q * Np + j] * xl[j];
            yr += Drc[q * Np + j] * yl[j];
            ys += Dsc[q * Np + j] * yl[j];
        }
        const double J = xr * ys - xs * yr;
        if (!(J > 0.0)) atomicAdd(count, 1);
        const double rx = ys / J, sx = -yr / J, ry = -xs / J, sy = xr / J;
        if (q == 0) {
            geoA[k * 5 + 0] = rx;
            geoA[k * 5 + 1] = sx;
            geoA[k * 5 + 2] = ry;
            geoA[k * 5 + 3] = sy;
            geoA[k * 5 + 4] = J;
        }
        if (mk) {
            const double wJ = wq[q] * J;
            double *gq = geoC + ((long)cs * NQ + q) * 4;
            gq[0] = wJ * rx;
            gq[1] = wJ * sx;
            gq[2] = wJ * ry;
            gq[3] = wJ * sy;
            for (int i = 0; i < Np; ++i)
                for (int j = 0; j < Np; ++j) mk[i * Np + j] += wJ * Icub[q * Np + i] * Icub[q * Np + j];
        }
    }
    for (int f = 0; f < 3; ++f)
        for (int g = 0; g < NG; ++g) {
            const double *dr = Drg + (f * NG + g) * Np, *ds = Dsg + (f * NG + g) * Np;
            double xr = 0, xs = 0, yr = 0, ys = 0;
            for (int j = 0; j < Np; ++j) {
                xr += dr[j] * xl[j];
                xs += ds[j] * xl[j];
                yr += dr[j] * yl[j];
                ys += ds[j] * yl[j];
            }
            double ax, ay;
            if (f == 0) {
                ax = yr;
                ay = -xr;
            } else if (f == 1) {
                ax = ys - yr;
                ay = xr - xs;
            } else {
                ax = -ys;
                ay = xs;
            }
            const double sJ = sqrt(ax * ax + ay * ay);
            double *gf = geoF + ((k * 3 + f) * NG + g) * 3;
            gf[0] = ax / sJ;
            gf[1] = ay / sJ;
            gf[2] = wg[g] * sJ;
        }
}

// Inverse of each curved element's mass matrix by Cholesky factorisation
// (M = L L^T, factor in `work`, then M^{-1} column by column from
// L y = e_i, L^T x = y), one thread per curved element, in FP64.
__global__ void k_weak_minv(int Kc, int Np, double *__restrict__ mass, double *__restrict__ work,
                            int *__restrict__ count) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= Kc) return;
    double *M = mass + c * Np * Np, *L = work + c * Np * Np;
    for (int z = 0; z < Np * Np; ++z) L[z] = 0.0;
    for (int j = 0; j < Np; ++j) {
        double d = M[j * Np + j];
        for (int k = 0; k < j; ++k) d -= L[j * Np + k] * L[j * Np + k];
        if (!(d > 0.0)) {
            atomicAdd(count, 1);
            return;
        }
        d = sqrt(d);
        L[j * Np + j] = d;
        for (int i = j + 1; i < Np; ++i) {
            double v = M[i * Np + j];
            for (int k = 0; k < j; ++k) v -= L[i * Np + k] * L[j * Np + k];
            L[i * Np + j] = v / d;
        }
    }
    for (int col = 0; col < Np; ++col) {
        // forward, into M's column col (M is no longer needed row-wise
        // beyond what the solve reads: the solve reads only L)
        for (int i = 0; i < Np; ++i) {
            double v = i == col ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= L[i * Np + k] * M[k * Np + col];
            M[i * Np + col] = v / L[i * Np + i];
        }
        for (int i = Np - 1; i >= 0; --i) {
            double v = M[i * Np + col];
            for (int k = i + 1; k < Np; ++k) v -= L[k * Np + i] * M[k * Np + col];
            M[i * Np + col] = v / L[i * Np + i];
        }
    }
}

template <typename F>
hipError_t with_order_w(int P, F &&f) {
    switch (P) {
        case 1: return f(std::integral_constant<int, 1>());
        case 2: return f(std::integral_constant<int, 2>());
        case 3: return f(std::integral_constant<int, 3>());
        case 4: return f(std::integral_constant<int, 4>());
        case 5: return f(std::integral_constant<int, 5>());
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t stage_weak_t(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                        hipStream_t st) {
    WeakArgs<T> a;
    a.K = m.K;
    a.stage = stage;
    a.mode = rhs ? 0 : 1;
    a.riemann = m.riemann;
    a.g = T(m.gamma);
    a.ra = T(rk_a(stage));
    a.rb = T(rk_b(stage));
    a.ff = make_farfield<T>(m.gamma, m.qinf);
    a.Uin = static_cast<const T *>(Uin);
    a.Uout = static_cast<T *>(Uout);
    a.R = static_cast<T *>(R);
    a.rhs = static_cast<T *>(rhs);
    a.nbr = m.nbr;
    a.finfo = m.finfo;
    if constexpr (sizeof(T) == 8) {
        a.ops = m.wops64;
        a.geoA = m.wgeoA64;
        a.geoF = m.wgeoF64;
        a.geoC = m.wgeoC64;
        a.minv = m.wminv64;
    } else {
        a.ops = m.wops32;
        a.geoA = m.wgeoA32;
        a.geoF = m.wgeoF32;
        a.geoC = m.wgeoC32;
        a.minv = m.wminv32;
    }
    a.widx = m.widx;
    a.dt = m.scal + S_DT;
    return with_order_w(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        constexpr int EB = weak_elems<T, P>();
        const dim3 grid(unsigned((m.K + EB - 1) / EB)), block(kWBlock);
        hipLaunchKernelGGL((k_stage_weak<T, P>), grid, block, 0, st, a);
        return hipGetLastError();
    });
}

}  // namespace

size_t weak_ops_size(int P) {
    const int Np = (P + 1) * (P + 2) / 2, Nfp = P + 1, n = (3 * P + 2) / 2, NQ = n * n;
    return size_t(3) * NQ * Np + NQ + size_t(n) * Nfp + size_t(Np) * Np;
}

hipError_t launch_weak_geometry(const DevMesh &m, const double *x, const double *y, const double *Drg,
                                const double *Dsg, const double *wg, double *geoA, double *geoF, double *geoC,
                                double *mass, double *work, hipStream_t st) {
    hipError_t e = with_order_w(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_weak_geometry<P>), dim3((m.K + 63) / 64), dim3(64), 0, st, m.K, x, y, m.wops64,
                           Drg, Dsg, wg, m.widx, geoA, geoF, geoC, mass, m.count);
        return hipGetLastError();
    });
    if (e != hipSuccess || m.wKc == 0) return e;
    hipLaunchKernelGGL(k_weak_minv, dim3((m.wKc + 63) / 64), dim3(64), 0, st, m.wKc, m.Np, mass, work,
                       m.count + 2);
    return hipGetLastError();
}

hipError_t launch_stage_weak(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                             hipStream_t st) {
    if (m.fp32 && m.wopsA) return launch_stage_weak_mfma(m, Uin, Uout, R, rhs, stage, st);
    return m.fp32 ? stage_weak_t<float>(m, Uin, Uout, R, rhs, stage, st)
                  : stage_weak_t<double>(m, Uin, Uout, R, rhs, stage, st);
}

}  // namespace dg
