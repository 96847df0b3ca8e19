// HIP kernels of the nodal DG Euler solver for gfx950 (VALU path).
//
// Tiling: one 64-lane wavefront holds EW = floor(64/Np) whole elements, one
// lane per node (lane = element * Np + node); a 256-thread block holds four
// wavefronts.  Elements never straddle wavefronts.  The element's state,
// fluxes and scaled face-flux jumps are staged in LDS; each lane keeps its
// own rows of Dr, Ds and LIFT in registers and forms the contractions
//   rhs_i = -(r_x (Dr F)_i + s_x (Ds F)_i + r_y (Dr G)_i + s_y (Ds G)_i)
//           + sum_q LIFT_iq Fscale_q (n.F(U-) - F*)_q
// (the semi-discrete system in nodal strong form), followed by the
// low-storage Runge-Kutta update in the same kernel.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstring>

#include "common.hpp"
#include "launch.hpp"

namespace dg {
namespace {

constexpr int kBlock = 256;

template <typename T>
struct StageArgs {
    int K, stage, mode;
    int riemann;   // numerical flux: RIEMANN_LF or RIEMANN_HLLC
    T g, ra, rb;
    FarField<T> ff;
    const T *__restrict__ Uin;
    T *__restrict__ Uout;
    T *__restrict__ R;
    T *__restrict__ rhs;
    const int *__restrict__ nbr;
    const int *__restrict__ finfo;
    const T *__restrict__ geo;
    const T *__restrict__ fgeo;
    const T *__restrict__ ops;
    const double *__restrict__ dt;
    const T *__restrict__ eps;
    const T *__restrict__ Q;
};

// Lane -> (local element, node) map shared by all element-tiled kernels.
template <int P>
struct Tile {
    using O = Order<P>;
    int lane, wave, le, i, el;
    long k;
    bool act;
    // tile `tile` of a mesh of K elements (a single-mesh launch: the block index)
    __device__ Tile(int K, int tile) {
        lane = threadIdx.x & 63;
        wave = threadIdx.x >> 6;
        le = lane / O::Np;
        i = lane - le * O::Np;
        bool lane_ok = le < O::EW;
        el = lane_ok ? wave * O::EW + le : 0;
        k = (long)tile * O::EB + wave * O::EW + le;
        act = lane_ok && k < K;
    }
    __device__ explicit Tile(int K) : Tile(K, blockIdx.x) {}
};

// A block-wide copy of N values into LDS in two halves: load() issues each
// thread's loads back to back (indices clamped, no branches) and store()
// writes them to LDS later, after the kernel has issued its own loads, so
// that the copy's latency overlaps theirs instead of preceding them.
template <typename T, int N>
struct LdsCopy {
    static constexpr int R = (N + kBlock - 1) / kBlock;
    T v[R];
    __device__ void load(const T *__restrict__ src) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[min(int(threadIdx.x) + r * kBlock, N - 1)];
    }
    __device__ void store(T *dst) const {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int z = int(threadIdx.x) + r * kBlock;
            if (z < N) dst[z] = v[r];
        }
    }
};

template <typename T, int P, bool AV>
__global__ __launch_bounds__(kBlock) void k_stage(StageArgs<T> a) {
    using O = Order<P>;
    constexpr int Np = O::Np, Nfp = O::Nfp, NF3 = O::Nface, EB = O::EB;
    __shared__ T sU[EB][kFields][Np];
    __shared__ T sF[EB][2 * kFields][Np];
    __shared__ T sJ[EB][kFields][NF3];
    // Dr, Ds and LIFT staged once per block; every thread needs its node's
    // rows of them, which through the caches cost a memory instruction per
    // entry
    constexpr int NOPS = 2 * Np * Np + Np * NF3;
    __shared__ T sOps[NOPS];
    LdsCopy<T, NOPS> opsc;
    opsc.load(a.ops);
    Tile<P> t(a.K);
    const long k = t.k;
    const int i = t.i, el = t.el;

    T u[kFields] = {};
    T sig = T(0);
    if (t.act) {
#pragma unroll
        for (int c = 0; c < kFields; ++c) u[c] = a.Uin[(k * kFields + c) * Np + i];
        T ir = rcp(u[0]);
        T vx = u[1] * ir, vy = u[2] * ir;
        T p = pressure_ir(a.g, u, ir);
        T F[kFields] = {u[1], u[1] * vx + p, u[2] * vx, (u[3] + p) * vx};
        T G[kFields] = {u[2], u[1] * vy, u[2] * vy + p, (u[3] + p) * vy};
        if (AV) {
            sig = sqrt(a.eps[k]);
#pragma unroll
            for (int c = 0; c < kFields; ++c) {
                F[c] -= sig * a.Q[((k * 2 + 0) * kFields + c) * Np + i];
                G[c] -= sig * a.Q[((k * 2 + 1) * kFields + c) * Np + i];
            }
        }
#pragma unroll
        for (int c = 0; c < kFields; ++c) {
            sU[el][c][i] = u[c];
            sF[el][c][i] = F[c];
            sF[el][kFields + c][i] = G[c];
        }
    }
    opsc.store(sOps);
    __syncthreads();

    if (t.act) {
        const int info = a.finfo[k];
        for (int q = i; q < NF3; q += Np) {
            const int f = q / Nfp, j = q - f * Nfp;
            const int vm = face_node(P, f, j);
            T um[kFields], up[kFields], d[kFields];
#pragma unroll
            for (int c = 0; c < kFields; ++c) um[c] = sU[el][c][vm];
            const T nx = a.fgeo[(k * 3 + 0) * NF3 + q];
            const T ny = a.fgeo[(k * 3 + 1) * NF3 + q];
            const T fs = a.fgeo[(k * 3 + 2) * NF3 + q];
            const int code = face_bc(info, f);
            long kn = -1;
            int vp = 0;
            if (code == BC_INTERIOR) {
                kn = a.nbr[k * 3 + f];
                vp = face_node(P, face_nbr_face(info, f), Nfp - 1 - j);
#pragma unroll
                for (int c = 0; c < kFields; ++c) up[c] = a.Uin[(kn * kFields + c) * Np + vp];
            } else {
                ghost_state(a.g, code, um, nx, ny, a.ff, up);
            }
            flux_jump(a.riemann, a.g, um, up, nx, ny, d);
            if (AV && code != BC_FARFIELD) {
                // (sigma Q)*.n - (sigma Q)-.n: the central value inside, the
                // mirror closure at a wall (wall_visc_jump), zero at the far
                // field (the element's own value)
                T vmv[kFields], vj[kFields];
#pragma unroll
                for (int c = 0; c < kFields; ++c)
                    vmv[c] = sig * (nx * a.Q[((k * 2 + 0) * kFields + c) * Np + vm] +
                                    ny * a.Q[((k * 2 + 1) * kFields + c) * Np + vm]);
                if (kn >= 0) {
                    const T sp = sqrt(a.eps[kn]);
#pragma unroll
                    for (int c = 0; c < kFields; ++c) {
                        T vpv = sp * (nx * a.Q[((kn * 2 + 0) * kFields + c) * Np + vp] +
                                      ny * a.Q[((kn * 2 + 1) * kFields + c) * Np + vp]);
                        vj[c] = T(0.5) * (vmv[c] + vpv) - vmv[c];
                    }
                } else {
                    wall_visc_jump(vmv, nx, ny, vj);
                }
#pragma unroll
                for (int c = 0; c < kFields; ++c) d[c] += vj[c];
            }
#pragma unroll
            for (int c = 0; c < kFields; ++c) sJ[el][c][q] = fs * d[c];
        }
    }
    __syncthreads();
    if (!t.act) return;

    // the node's operator rows: copied into registers up to P = 4; at P = 5
    // (60 values) read from LDS inside the contraction, which leaves the
    // registers for more resident waves (faster there, slower below; the
    // values and the order of operations are the same either way)
    constexpr bool kRowsInRegs = P < 5;
    T rdr[kRowsInRegs ? Np : 1], rds[kRowsInRegs ? Np : 1], rlf[kRowsInRegs ? NF3 : 1];
    if constexpr (kRowsInRegs) {
#pragma unroll
        for (int j = 0; j < Np; ++j) {
            rdr[j] = sOps[i * Np + j];
            rds[j] = sOps[Np * Np + i * Np + j];
        }
#pragma unroll
        for (int q = 0; q < NF3; ++q) rlf[q] = sOps[2 * Np * Np + i * NF3 + q];
    }
    auto dr = [&](int j) -> T {
        if constexpr (kRowsInRegs) return rdr[j]; else return sOps[i * Np + j];
    };
    auto ds = [&](int j) -> T {
        if constexpr (kRowsInRegs) return rds[j]; else return sOps[Np * Np + i * Np + j];
    };
    auto lf = [&](int q) -> T {
        if constexpr (kRowsInRegs) return rlf[q]; else return sOps[2 * Np * Np + i * NF3 + q];
    };
    const T rx = a.geo[(k * 4 + 0) * Np + i], sx = a.geo[(k * 4 + 1) * Np + i];
    const T ry = a.geo[(k * 4 + 2) * Np + i], sy = a.geo[(k * 4 + 3) * Np + i];
    const T dt = a.mode ? T(*a.dt) : T(0);
    // at P = 5 the contractions run node by node across the four fields, so
    // that each operator entry is read from LDS once for all of them (the
    // same sums in the same order as field by field)
    T vol[kRowsInRegs ? 1 : kFields], lift[kRowsInRegs ? 1 : kFields];
    if constexpr (!kRowsInRegs) {
        T drf[kFields] = {}, dsf[kFields] = {}, drg[kFields] = {}, dsg[kFields] = {};
#pragma unroll 3
        for (int j = 0; j < Np; ++j) {
            const T dj = dr(j), sj = ds(j);
#pragma unroll
            for (int c = 0; c < kFields; ++c) {
                const T fv = sF[el][c][j], gv = sF[el][kFields + c][j];
                drf[c] += dj * fv;
                dsf[c] += sj * fv;
                drg[c] += dj * gv;
                dsg[c] += sj * gv;
            }
        }
#pragma unroll
        for (int c = 0; c < kFields; ++c) {
            vol[c] = -(rx * drf[c] + sx * dsf[c] + ry * drg[c] + sy * dsg[c]);
            lift[c] = vol[c];
        }
#pragma unroll 3
        for (int q = 0; q < NF3; ++q) {
            const T l = lf(q);
#pragma unroll
            for (int c = 0; c < kFields; ++c) lift[c] += l * sJ[el][c][q];
        }
    }
#pragma unroll
    for (int c = 0; c < kFields; ++c) {
        T val;
        if constexpr (!kRowsInRegs) {
            val = lift[c];
        } else {
            T drf = 0, dsf = 0, drg = 0, dsg = 0;
#pragma unroll
            for (int j = 0; j < Np; ++j) {
                const T fv = sF[el][c][j], gv = sF[el][kFields + c][j];
                drf += dr(j) * fv;
                dsf += ds(j) * fv;
                drg += dr(j) * gv;
                dsg += ds(j) * gv;
            }
            val = -(rx * drf + sx * dsf + ry * drg + sy * dsg);
#pragma unroll
            for (int q = 0; q < NF3; ++q) val += lf(q) * sJ[el][c][q];
        }
        const long idx = (k * kFields + c) * Np + i;
        if (a.mode == 0) {
            a.rhs[idx] = val;
        } else {
            T r = (a.stage == 0) ? dt * val : a.ra * a.R[idx] + dt * val;
            a.R[idx] = r;
            a.Uout[idx] = u[c] + a.rb * r;
        }
    }
}

// ---------------------------------------------------------------------------
// artificial viscosity
// ---------------------------------------------------------------------------

template <typename T>
struct AvArgs {
    int K, P;
    T g;
    double gamma;   // the time-step bound is formed in FP64
    FarField<T> ff;
    double s0, kappa;
    const T *__restrict__ U;
    const T *__restrict__ eps_in;
    T *__restrict__ eps_out;
    T *__restrict__ Q;
    const int *__restrict__ nbr;
    const int *__restrict__ finfo;
    const T *__restrict__ geo;
    const T *__restrict__ fgeo;
    const T *__restrict__ ops;
    const T *__restrict__ emax;
    unsigned long long *__restrict__ vmax;   // CFL-bound slots (sensor with the bound only)
    int *__restrict__ flag;                  // state check (sensor with the bound only)
};

// Persson-Peraire sensor on the density: u_hat = V^{-1} rho, S = (energy of
// the degree-P modes) / (total modal energy), s = log10 S, sine ramp of
// half-width kappa around s0, capped at eps_max,k.  CFL: also the time-step
// bound of the state with its new viscosity (FP64 per face node, cfl_bound),
// reduced into the block's slot, and the state check (rho, p > 0, finite).
template <typename T, int P, bool CFL>
__device__ __forceinline__ void sensor_body(const AvArgs<T> &a, const int tile) {
    using O = Order<P>;
    constexpr int Np = O::Np, Nfp = O::Nfp, NF3 = O::Nface, EB = O::EB;
    __shared__ T sR[EB][Np];
    __shared__ double sE[EB][Np];
    __shared__ T sEps[EB];
    __shared__ double sRed[kBlock / 64];
    // V^{-1} staged once per block: every thread reads a row of it, and
    // reading it through the caches costs a memory instruction per entry
    __shared__ T sVi[Np * Np];
    LdsCopy<T, Np * Np> vic;
    vic.load(a.ops + (2 * Np * Np + Np * 3 * Nfp));
    Tile<P> t(a.K, tile);
    if (t.act) sR[t.el][t.i] = a.U[(t.k * kFields + 0) * Np + t.i];
    vic.store(sVi);
    __syncthreads();
    if (t.act) {
        T uh = 0;
#pragma unroll
        for (int j = 0; j < Np; ++j) uh += sVi[t.i * Np + j] * sR[t.el][j];
        sE[t.el][t.i] = double(uh) * double(uh);
    }
    __syncthreads();
    if (t.act && t.i == 0) {
        double num = 0, den = 0;
#pragma unroll
        for (int j = 0; j < Np; ++j) {
            den += sE[t.el][j];
            if (j >= Np - Nfp) num += sE[t.el][j];
        }
        double emax = double(a.emax[t.k]);
        double e = 0.0;
        if (den > 1e-300 && num > 0.0) {
            double sk = log10(num / den);
            if (sk > a.s0 + a.kappa)
                e = emax;
            else if (sk >= a.s0 - a.kappa)
                e = 0.5 * emax * (1.0 + sin(M_PI * (sk - a.s0) / (2.0 * a.kappa)));
        }
        a.eps_out[t.k] = T(e);
        if constexpr (CFL) sEps[t.el] = T(e);
    }
    if constexpr (CFL) {
        __syncthreads();
        double vmax = 0.0;
        int bad = 0;
        if (t.act) {
            const T *Uk = a.U + t.k * kFields * Np;
            {
                double u[kFields];
#pragma unroll
                for (int c = 0; c < kFields; ++c) u[c] = double(Uk[c * Np + t.i]);
                if (bad_state(a.gamma, u)) bad = 1;
            }
            const double P1 = P + 1.0, e = double(sEps[t.el]);
            for (int q = t.i; q < NF3; q += Np) {
                const int v = face_node(P, q / Nfp, q % Nfp);
                double u[kFields];
#pragma unroll
                for (int c = 0; c < kFields; ++c) u[c] = double(Uk[c * Np + v]);
                const double val = cfl_bound(a.gamma, u, double(a.fgeo[(t.k * 3 + 2) * NF3 + q]), e, P1);
                vmax = val > vmax ? val : vmax;
            }
        }
        if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(a.flag, 1);
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(vmax, off);
            vmax = o > vmax ? o : vmax;
        }
        if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = vmax;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = sRed[0];
            for (int w = 1; w < kBlock / 64; ++w) m = sRed[w] > m ? sRed[w] : m;
            // non-negative doubles order like their bit patterns
            atomicMax(a.vmax + (blockIdx.x & (kVmaxSlots - 1)), (unsigned long long)__double_as_longlong(m));
        }
    }
}

template <typename T, int P, bool CFL>
__global__ __launch_bounds__(kBlock) void k_sensor(AvArgs<T> a) {
    sensor_body<T, P, CFL>(a, blockIdx.x);
}

// The sensor alone (no time-step bound) with one thread per element: the
// block copies the densities of its kBlock elements into LDS (contiguous
// runs of Np values, all loads issued before the first wait), then each
// thread forms its element's modal energies and viscosity with the same
// operations in the same order as sensor_body, so the results are the same
// bits, without the two block-wide phases per element.
template <typename T, int P>
__device__ __forceinline__ void sensor_elem_body(const AvArgs<T> &a, const int tile) {
    using O = Order<P>;
    constexpr int Np = O::Np, Nfp = O::Nfp;
    // an odd row stride puts the threads' rows in distinct LDS banks (Np is
    // even for P = 2, 3 and odd otherwise)
    constexpr int NR = Np | 1;
    __shared__ T sVi[Np * Np];
    __shared__ T sR[kBlock * NR];
    LdsCopy<T, Np * Np> vic;
    vic.load(a.ops + (2 * Np * Np + Np * 3 * Nfp));
    const long k0 = (long)tile * kBlock;
    const int nel = (int)min((long)kBlock, (long)a.K - k0);
    const int nval = nel * Np;
    T rv[Np];
#pragma unroll
    for (int r = 0; r < Np; ++r) {
        const int z = min(int(threadIdx.x) + r * kBlock, nval - 1);
        const int e = z / Np, j = z - e * Np;
        rv[r] = a.U[(k0 + e) * kFields * Np + j];
    }
#pragma unroll
    for (int r = 0; r < Np; ++r) {
        const int z = int(threadIdx.x) + r * kBlock;
        if (z < nval) {
            const int e = z / Np, j = z - e * Np;
            sR[e * NR + j] = rv[r];
        }
    }
    vic.store(sVi);
    __syncthreads();
    if (int(threadIdx.x) >= nel) return;
    const long k = k0 + threadIdx.x;
    const T emax_k = a.emax[k];
    T rho[Np];
#pragma unroll
    for (int j = 0; j < Np; ++j) rho[j] = sR[threadIdx.x * NR + j];
    double num = 0, den = 0;
#pragma unroll
    for (int i = 0; i < Np; ++i) {
        T uh = 0;
#pragma unroll
        for (int j = 0; j < Np; ++j) uh += sVi[i * Np + j] * rho[j];
        const double e2 = double(uh) * double(uh);
        den += e2;
        if (i >= Np - Nfp) num += e2;
    }
    double emax = double(emax_k);
    double e = 0.0;
    if (den > 1e-300 && num > 0.0) {
        double sk = log10(num / den);
        if (sk > a.s0 + a.kappa)
            e = emax;
        else if (sk >= a.s0 - a.kappa)
            e = 0.5 * emax * (1.0 + sin(M_PI * (sk - a.s0) / (2.0 * a.kappa)));
    }
    a.eps_out[k] = T(e);
}

template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_sensor_elem(AvArgs<T> a) {
    sensor_elem_body<T, P>(a, blockIdx.x);
}

// Auxiliary variable of the viscous system, q = sigma grad U (sigma =
// sqrt eps_k), strong form with the central trace (sigma U)*:
//   Q_x = sigma (r_x Dr U + s_x Ds U) + LIFT [Fscale n_x ((sigma U)* - sigma U-)]
template <typename T, int P>
__device__ __forceinline__ void avgrad_body(const AvArgs<T> &a, const int tile) {
    using O = Order<P>;
    constexpr int Np = O::Np, Nfp = O::Nfp, NF3 = O::Nface, EB = O::EB;
    __shared__ T sU[EB][kFields][Np];
    __shared__ T sX[EB][kFields][NF3];
    __shared__ T sY[EB][kFields][NF3];
    // Dr, Ds and LIFT staged once per block (the same values in the same
    // order as from global memory, so the results do not change; the block
    // then reads them from LDS instead of issuing a cached load per entry)
    constexpr int NOPS = 2 * Np * Np + Np * NF3;
    __shared__ T sOps[NOPS];
    LdsCopy<T, NOPS> opsc;
    opsc.load(a.ops);
    Tile<P> t(a.K, tile);
    const long k = t.k;
    const int i = t.i, el = t.el;
    T sig = 0;
    if (t.act) {
        sig = sqrt(a.eps_in[k]);
#pragma unroll
        for (int c = 0; c < kFields; ++c) sU[el][c][i] = a.U[(k * kFields + c) * Np + i];
    }
    opsc.store(sOps);
    __syncthreads();
    if (t.act) {
        const int info = a.finfo[k];
        for (int q = i; q < NF3; q += Np) {
            const int f = q / Nfp, j = q - f * Nfp;
            const int vm = face_node(P, f, j);
            T um[kFields], up[kFields];
#pragma unroll
            for (int c = 0; c < kFields; ++c) um[c] = sU[el][c][vm];
            const T nx = a.fgeo[(k * 3 + 0) * NF3 + q];
            const T ny = a.fgeo[(k * 3 + 1) * NF3 + q];
            const T fs = a.fgeo[(k * 3 + 2) * NF3 + q];
            const int code = face_bc(info, f);
            T sp = sig;
            if (code == BC_INTERIOR) {
                const long kn = a.nbr[k * 3 + f];
                const int vp = face_node(P, face_nbr_face(info, f), Nfp - 1 - j);
                sp = sqrt(a.eps_in[kn]);
#pragma unroll
                for (int c = 0; c < kFields; ++c) up[c] = a.U[(kn * kFields + c) * Np + vp];
            } else {
                ghost_state(a.g, code, um, nx, ny, a.ff, up);
            }
#pragma unroll
            for (int c = 0; c < kFields; ++c) {
                T star = T(0.5) * (sig * um[c] + sp * up[c]);
                T d = fs * (star - sig * um[c]);
                sX[el][c][q] = nx * d;
                sY[el][c][q] = ny * d;
            }
        }
    }
    __syncthreads();
    if (!t.act) return;
    const T rx = a.geo[(k * 4 + 0) * Np + i], sx = a.geo[(k * 4 + 1) * Np + i];
    const T ry = a.geo[(k * 4 + 2) * Np + i], sy = a.geo[(k * 4 + 3) * Np + i];
#pragma unroll
    for (int c = 0; c < kFields; ++c) {
        T dru = 0, dsu = 0;
#pragma unroll
        for (int j = 0; j < Np; ++j) {
            const T uv = sU[el][c][j];
            dru += sOps[i * Np + j] * uv;
            dsu += sOps[Np * Np + i * Np + j] * uv;
        }
        T qx = sig * (rx * dru + sx * dsu);
        T qy = sig * (ry * dru + sy * dsu);
#pragma unroll
        for (int q = 0; q < NF3; ++q) {
            const T l = sOps[2 * Np * Np + i * NF3 + q];
            qx += l * sX[el][c][q];
            qy += l * sY[el][c][q];
        }
        a.Q[((k * 2 + 0) * kFields + c) * Np + i] = qx;
        a.Q[((k * 2 + 1) * kFields + c) * Np + i] = qy;
    }
}

template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_avgrad(AvArgs<T> a) {
    avgrad_body<T, P>(a, blockIdx.x);
}

// Batched meshes of one order (FP32 viscous handles): work item = (job,
// tile), a job being one mesh's argument record for this stage.
// One work item per block; the grid covers the list's capacity and the
// length is read from device memory (a captured launch stays valid when the
// list changes); surplus blocks exit.
template <int P, bool CFL>
__global__ __launch_bounds__(kBlock) void k_sensor_batch(const AvArgs<float> *__restrict__ jobs,
                                                         const int2 *__restrict__ items,
                                                         const int *__restrict__ nitems_dev) {
    const int w = int(blockIdx.x);
    if (w >= *nitems_dev) return;
    const int2 it = items[w];
    sensor_body<float, P, CFL>(jobs[it.x], it.y);
}

// Batched per-element sensor: work item = (job, block of kBlock elements).
template <int P>
__global__ __launch_bounds__(kBlock) void k_sensor_elem_batch(const AvArgs<float> *__restrict__ jobs,
                                                              const int2 *__restrict__ items,
                                                              const int *__restrict__ nitems_dev) {
    const int w = int(blockIdx.x);
    if (w >= *nitems_dev) return;
    const int2 it = items[w];
    sensor_elem_body<float, P>(jobs[it.x], it.y);
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_avgrad_batch(const AvArgs<float> *__restrict__ jobs,
                                                         const int2 *__restrict__ items,
                                                         const int *__restrict__ nitems_dev) {
    const int w = int(blockIdx.x);
    if (w >= *nitems_dev) return;
    const int2 it = items[w];
    avgrad_body<float, P>(jobs[it.x], it.y);
}

// ---------------------------------------------------------------------------
// geometry (FP64, once per mesh)
// ---------------------------------------------------------------------------

template <int P>
__global__ __launch_bounds__(kBlock) void k_geometry(int K, const double *__restrict__ x,
                                                     const double *__restrict__ y,
                                                     const double *__restrict__ ops,
                                                     const double *__restrict__ Mref,
                                                     double *__restrict__ geo,
                                                     double *__restrict__ fgeo,
                                                     double *__restrict__ wmass,
                                                     double *__restrict__ emax, double av_eps0,
                                                     int *__restrict__ count) {
    using O = Order<P>;
    constexpr int Np = O::Np, Nfp = O::Nfp, NF3 = O::Nface, EB = O::EB;
    __shared__ double sX[EB][Np], sY[EB][Np], sJ[EB][Np];
    __shared__ double sM[EB][4][Np];  // xr, xs, yr, ys
    __shared__ double sFs[EB][NF3];
    Tile<P> t(K);
    const long k = t.k;
    const int i = t.i, el = t.el;
    // coordinates relative to the element's first node: Dr and Ds annihilate
    // constants, so the metric terms are the same in exact arithmetic, but
    // the sums no longer cancel the absolute position (on small elements far
    // from the origin that cancellation costs ~|x| / h of the metric terms'
    // precision)
    if (t.act) {
        sX[el][i] = x[k * Np + i] - x[k * Np];
        sY[el][i] = y[k * Np + i] - y[k * Np];
    }
    __syncthreads();
    if (t.act) {
        double xr = 0, xs = 0, yr = 0, ys = 0;
        for (int j = 0; j < Np; ++j) {
            const double dr = ops[i * Np + j], ds = ops[Np * Np + i * Np + j];
            xr += dr * sX[el][j];
            xs += ds * sX[el][j];
            yr += dr * sY[el][j];
            ys += ds * sY[el][j];
        }
        const double J = xr * ys - xs * yr;
        if (!(J > 0.0)) atomicAdd(count, 1);
        geo[(k * 4 + 0) * Np + i] = ys / J;
        geo[(k * 4 + 1) * Np + i] = -yr / J;
        geo[(k * 4 + 2) * Np + i] = -xs / J;
        geo[(k * 4 + 3) * Np + i] = xr / J;
        sJ[el][i] = J;
        sM[el][0][i] = xr;
        sM[el][1][i] = xs;
        sM[el][2][i] = yr;
        sM[el][3][i] = ys;
    }
    __syncthreads();
    if (t.act) {
        for (int q = i; q < NF3; q += Np) {
            const int f = q / Nfp, j = q - f * Nfp;
            const int v = face_node(P, f, j);
            const double xr = sM[el][0][v], xs = sM[el][1][v], yr = sM[el][2][v], ys = sM[el][3][v];
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
            const double len = sqrt(ax * ax + ay * ay);
            fgeo[(k * 3 + 0) * NF3 + q] = ax / len;
            fgeo[(k * 3 + 1) * NF3 + q] = ay / len;
            const double fsc = len / sJ[el][v];
            fgeo[(k * 3 + 2) * NF3 + q] = fsc;
            sFs[el][q] = fsc;
        }
        double w = 0;
        for (int j = 0; j < Np; ++j) w += Mref[i * Np + j] * sJ[el][j];
        wmass[k * Np + i] = w;
    }
    __syncthreads();
    if (t.act && i == 0) {
        double fmax = 0;
        for (int q = 0; q < NF3; ++q) fmax = fmax > sFs[el][q] ? fmax : sFs[el][q];
        emax[k] = av_eps0 * (2.0 / fmax) / P;
    }
}

template <int P>
__global__ void k_check_normals(int K, const int *__restrict__ nbr, const int *__restrict__ finfo,
                                const double *__restrict__ fgeo, int *__restrict__ count) {
    constexpr int Nfp = P + 1, NF3 = 3 * Nfp;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long)K * NF3) return;
    const long k = gid / NF3;
    const int q = int(gid - k * NF3);
    const int f = q / Nfp, j = q - f * Nfp;
    const int info = finfo[k];
    if (face_bc(info, f) != BC_INTERIOR) return;
    const long kn = nbr[k * 3 + f];
    const int qn = face_nbr_face(info, f) * Nfp + Nfp - 1 - j;
    const double ex = fgeo[(k * 3 + 0) * NF3 + q] + fgeo[(kn * 3 + 0) * NF3 + qn];
    const double ey = fgeo[(k * 3 + 1) * NF3 + q] + fgeo[(kn * 3 + 1) * NF3 + qn];
    if (!(fabs(ex) <= 1e-10 && fabs(ey) <= 1e-10)) atomicAdd(count + 1, 1);
}

template <int P>
__global__ void k_affine_flags(int K, const double *__restrict__ geo, const double *__restrict__ fgeo,
                               int *__restrict__ flags) {
    constexpr int Np = (P + 1) * (P + 2) / 2, Nfp = P + 1, NF3 = 3 * Nfp;
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    bool affine = true;
    // one scale for the four metric terms: a term that is near zero on this
    // element (an edge nearly parallel to an axis) varies by the rounding of
    // the others, which relative to itself can be large
    double scale = 0;
    for (int m = 0; m < 4; ++m)
        for (int i = 0; i < Np; ++i) scale = fmax(scale, fabs(geo[(k * 4 + m) * Np + i]));
    for (int m = 0; m < 4; ++m) {
        const double *g = geo + (k * 4 + m) * Np;
        for (int i = 1; i < Np; ++i) affine &= fabs(g[i] - g[0]) <= 1e-10 * scale;
    }
    for (int m = 0; m < 3; ++m) {
        const double *g = fgeo + (k * 3 + m) * NF3;
        for (int f = 0; f < 3; ++f) {
            const double ref = g[f * Nfp];
            const double scale = m == 2 ? fabs(ref) : 1.0;
            for (int j = 1; j < Nfp; ++j) affine &= fabs(g[f * Nfp + j] - ref) <= 1e-10 * scale;
        }
    }
    flags[k] = affine ? 1 : 0;
}

template <int P>
__global__ void k_pack_geometry(int K, const double *__restrict__ geo, const double *__restrict__ fgeo,
                                const int *__restrict__ cidx, float *__restrict__ geoA,
                                float *__restrict__ geoC) {
    constexpr int Np = (P + 1) * (P + 2) / 2, Nfp = P + 1, NF3 = 3 * Nfp;
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    float *ga = geoA + k * 16;
    for (int m = 0; m < 4; ++m) ga[m] = float(geo[(k * 4 + m) * Np]);
    for (int f = 0; f < 3; ++f)
        for (int m = 0; m < 3; ++m) ga[4 + 3 * f + m] = float(fgeo[(k * 3 + m) * NF3 + f * Nfp]);
    const int c = cidx[k];
    // slot 13: 1 for a curved element (its per-node record is in geoC)
    ga[13] = c >= 0 ? 1.f : 0.f;
    ga[14] = ga[15] = 0.f;
    if (c >= 0) {
        float *gc = geoC + (long)c * (4 * Np + 9 * Nfp);
        for (int m = 0; m < 4; ++m)
            for (int i = 0; i < Np; ++i) gc[m * Np + i] = float(geo[(k * 4 + m) * Np + i]);
        for (int m = 0; m < 3; ++m)
            for (int q = 0; q < NF3; ++q) gc[4 * Np + m * NF3 + q] = float(fgeo[(k * 3 + m) * NF3 + q]);
    }
}

__global__ void k_cast(const double *__restrict__ src, float *__restrict__ dst, size_t n) {
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) dst[g] = float(src[g]);
}

template <typename T>
__global__ void k_eps_to_double(const T *__restrict__ src, double *__restrict__ dst, int n) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) dst[g] = double(src[g]);
}

// ---------------------------------------------------------------------------
// FP64 reductions: time step, totals, residual
// ---------------------------------------------------------------------------

// Fixed-shape tree reduction over the block (deterministic).
template <typename Op>
__device__ double block_reduce(double v, double *sh, Op op) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = op(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

struct MaxOp {
    __device__ double operator()(double a, double b) const { return a > b ? a : b; }
};
struct SumOp {
    __device__ double operator()(double a, double b) const { return a + b; }
};

template <typename T, int P, bool AV>
__global__ __launch_bounds__(kBlock) void k_cfl(int K, double g, const T *__restrict__ U,
                                                const T *__restrict__ eps,
                                                const double *__restrict__ fgeo64,
                                                double *__restrict__ partial,
                                                int *__restrict__ flag) {
    using O = Order<P>;
    constexpr int Np = O::Np, Nfp = O::Nfp, NF3 = O::Nface, EB = O::EB;
    __shared__ double sU[EB][kFields][Np];
    __shared__ double sh[kBlock];
    Tile<P> t(K);
    const long k = t.k;
    const int i = t.i, el = t.el;
    int bad = 0;
    if (t.act) {
        double u[kFields];
#pragma unroll
        for (int c = 0; c < kFields; ++c) {
            u[c] = double(U[(k * kFields + c) * Np + i]);
            sU[el][c][i] = u[c];
        }
        if (bad_state(g, u)) bad = 1;
    }
    __syncthreads();
    double vmax = 0.0;
    if (t.act) {
        const double P1 = P + 1.0;
        const double e = AV ? double(eps[k]) : 0.0;
        for (int q = i; q < NF3; q += Np) {
            const int f = q / Nfp, j = q - f * Nfp;
            const int v = face_node(P, f, j);
            double u[kFields];
#pragma unroll
            for (int c = 0; c < kFields; ++c) u[c] = sU[el][c][v];
            const double val = cfl_bound(g, u, fgeo64[(k * 3 + 2) * NF3 + q], e, P1);
            if (val > vmax) vmax = val;
        }
    }
    if (bad) atomicOr(flag, 1);
    const double r = block_reduce(vmax, sh, MaxOp());
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ __launch_bounds__(kBlock) void k_cfl_finish(int n, const double *__restrict__ partial,
                                                       double cfl, double dt_fixed,
                                                       double *__restrict__ scal) {
    __shared__ double sh[kBlock];
    double v = 0.0;
    // unrolled so that eight loads are in flight per wait (the maximum is
    // exact in any order)
#pragma unroll 8
    for (int b = threadIdx.x; b < n; b += kBlock) v = v > partial[b] ? v : partial[b];
    const double vmax = block_reduce(v, sh, MaxOp());
    if (threadIdx.x == 0) {
        const double dt = dt_fixed > 0.0 ? dt_fixed : cfl * (1.0 / vmax);
        scal[S_DT] = dt;
        scal[S_T] += dt;
        scal[S_DTMIN] = dt < scal[S_DTMIN] ? dt : scal[S_DTMIN];
        scal[S_DTMAX] = dt > scal[S_DTMAX] ? dt : scal[S_DTMAX];
        scal[S_STEPS] += 1.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_cfl_finish_vmax(int n, const double *__restrict__ partial,
                                                            unsigned long long *__restrict__ slot) {
    __shared__ double sh[kBlock];
    double v = 0.0;
#pragma unroll 8
    for (int b = threadIdx.x; b < n; b += kBlock) v = v > partial[b] ? v : partial[b];
    const double vmax = block_reduce(v, sh, MaxOp());
    // the bound in the first slot, zeros in the others
    if (threadIdx.x < kVmaxSlots)
        slot[threadIdx.x] = threadIdx.x == 0 ? (unsigned long long)__double_as_longlong(vmax) : 0ull;
}

template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_totals(int K, const T *__restrict__ U,
                                                   const double *__restrict__ wmass,
                                                   double *__restrict__ partial) {
    using O = Order<P>;
    constexpr int Np = O::Np;
    __shared__ double sh[kBlock];
    Tile<P> t(K);
    double v[kFields] = {0, 0, 0, 0};
    if (t.act) {
        const double w = wmass[t.k * Np + t.i];
#pragma unroll
        for (int c = 0; c < kFields; ++c) v[c] = w * double(U[(t.k * kFields + c) * Np + t.i]);
    }
#pragma unroll
    for (int c = 0; c < kFields; ++c) {
        const double r = block_reduce(v[c], sh, SumOp());
        if (threadIdx.x == 0) partial[blockIdx.x * kFields + c] = r;
    }
}

template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_absmax(int K, const T *__restrict__ X,
                                                   double *__restrict__ partial) {
    using O = Order<P>;
    constexpr int Np = O::Np;
    __shared__ double sh[kBlock];
    Tile<P> t(K);
    double v[kFields] = {0, 0, 0, 0};
    if (t.act) {
#pragma unroll
        for (int c = 0; c < kFields; ++c) v[c] = fabs(double(X[(t.k * kFields + c) * Np + t.i]));
    }
#pragma unroll
    for (int c = 0; c < kFields; ++c) {
        const double r = block_reduce(v[c], sh, MaxOp());
        if (threadIdx.x == 0) partial[blockIdx.x * kFields + c] = r;
    }
}

template <typename Op>
__global__ __launch_bounds__(kBlock) void k_finish4(int n, const double *__restrict__ partial,
                                                    double *__restrict__ out, Op op) {
    __shared__ double sh[kBlock];
    for (int c = 0; c < kFields; ++c) {
        double v = 0.0;
        for (int b = threadIdx.x; b < n; b += kBlock) v = op(v, partial[b * kFields + c]);
        const double r = block_reduce(v, sh, op);
        if (threadIdx.x == 0) out[c] = r;
    }
}

__global__ void k_reset_scalars(double *scal) {
    if (threadIdx.x == 0) {
        for (int s = 0; s < S_NSCAL; ++s) scal[s] = 0.0;
        scal[S_DTMIN] = DBL_MAX;
    }
}

// ---------------------------------------------------------------------------
// dispatch helpers
// ---------------------------------------------------------------------------

template <int P>
int nblocks(int K) {
    return (K + Order<P>::EB - 1) / Order<P>::EB;
}

int nblocks_rt(int K, int P) {
    switch (P) {
        case 1: return nblocks<1>(K);
        case 2: return nblocks<2>(K);
        case 3: return nblocks<3>(K);
        case 4: return nblocks<4>(K);
        default: return nblocks<5>(K);
    }
}

template <typename F>
hipError_t with_order(int P, F &&f) {
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
const T *tbl_geo(const DevMesh &m);
template <>
const double *tbl_geo<double>(const DevMesh &m) { return m.geo64; }
template <>
const float *tbl_geo<float>(const DevMesh &m) { return m.geo32; }
template <typename T>
const T *tbl_fgeo(const DevMesh &m);
template <>
const double *tbl_fgeo<double>(const DevMesh &m) { return m.fgeo64; }
template <>
const float *tbl_fgeo<float>(const DevMesh &m) { return m.fgeo32; }
template <typename T>
const T *tbl_ops(const DevMesh &m);
template <>
const double *tbl_ops<double>(const DevMesh &m) { return m.ops64; }
template <>
const float *tbl_ops<float>(const DevMesh &m) { return m.ops32; }
template <typename T>
const T *tbl_emax(const DevMesh &m);
template <>
const double *tbl_emax<double>(const DevMesh &m) { return m.emax64; }
template <>
const float *tbl_emax<float>(const DevMesh &m) { return m.emax32; }

template <typename T>
hipError_t stage_t(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                   const void *eps, const void *Q, hipStream_t st) {
    StageArgs<T> a;
    a.riemann = m.riemann;
    a.K = m.K;
    a.stage = stage;
    a.mode = rhs ? 0 : 1;
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
    a.geo = tbl_geo<T>(m);
    a.fgeo = tbl_fgeo<T>(m);
    a.ops = tbl_ops<T>(m);
    a.dt = m.scal + S_DT;
    a.eps = static_cast<const T *>(eps);
    a.Q = static_cast<const T *>(Q);
    return with_order(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        if (m.av)
            hipLaunchKernelGGL((k_stage<T, P, true>), dim3(nblocks<P>(m.K)), dim3(kBlock), 0, st, a);
        else
            hipLaunchKernelGGL((k_stage<T, P, false>), dim3(nblocks<P>(m.K)), dim3(kBlock), 0, st, a);
        return hipGetLastError();
    });
}

template <typename T>
AvArgs<T> av_args(const DevMesh &m) {
    AvArgs<T> a;
    a.K = m.K;
    a.P = m.P;
    a.g = T(m.gamma);
    a.gamma = m.gamma;
    a.ff = make_farfield<T>(m.gamma, m.qinf);
    a.s0 = m.av_s0;
    a.kappa = m.av_kappa;
    a.nbr = m.nbr;
    a.finfo = m.finfo;
    a.geo = tbl_geo<T>(m);
    a.fgeo = tbl_fgeo<T>(m);
    a.ops = tbl_ops<T>(m);
    a.emax = tbl_emax<T>(m);
    a.vmax = nullptr;
    a.flag = m.flag;
    return a;
}

}  // namespace

int partial_slots(int K, int P) { return nblocks_rt(K, P); }

hipError_t launch_geometry(const DevMesh &m, const double *x, const double *y, double *geo64,
                           double *fgeo64, double *wmass, double *emax64, double av_eps0,
                           hipStream_t st) {
    const double *Mref = m.ops64 + ops_size(m.Np, m.Nfp);
    return with_order(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_geometry<P>), dim3(nblocks<P>(m.K)), dim3(kBlock), 0, st, m.K, x, y,
                           m.ops64, Mref, geo64, fgeo64, wmass, emax64, av_eps0, m.count);
        return hipGetLastError();
    });
}

hipError_t launch_check_normals(const DevMesh &m, hipStream_t st) {
    return with_order(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        const long n = (long)m.K * 3 * (P + 1);
        hipLaunchKernelGGL((k_check_normals<P>), dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                           m.K, m.nbr, m.finfo, m.fgeo64, m.count);
        return hipGetLastError();
    });
}

hipError_t launch_affine_flags(const DevMesh &m, int *flags, hipStream_t st) {
    return with_order(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_affine_flags<P>), dim3((m.K + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                           m.K, m.geo64, m.fgeo64, flags);
        return hipGetLastError();
    });
}

hipError_t launch_pack_geometry(const DevMesh &m, const int *cidx, float *geoA, float *geoC,
                                hipStream_t st) {
    return with_order(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_pack_geometry<P>), dim3((m.K + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                           m.K, m.geo64, m.fgeo64, cidx, geoA, geoC);
        return hipGetLastError();
    });
}

hipError_t launch_cast(const double *src, float *dst, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cast, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_stage(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                        const void *eps, const void *Q, hipStream_t st) {
    // the weak form: its own kernel; FP32 (with or without viscosity): the
    // matrix-core kernel; FP64: the FP64 matrix cores for a mesh of straight
    // elements without viscosity, else VALU
    if (m.weak) return launch_stage_weak(m, Uin, Uout, R, rhs, stage, st);
    if (m.fp32) return launch_stage_mfma(m, Uin, Uout, R, rhs, stage, MfmaStep(), st, eps, Q);
    if (m.opsA64 && !m.av) return launch_stage_mfma64(m, Uin, Uout, R, rhs, stage, false, st);
    return stage_t<double>(m, Uin, Uout, R, rhs, stage, eps, Q, st);
}

template <typename T>
static hipError_t sensor_t(const DevMesh &m, const void *U, void *eps, unsigned long long *vmax,
                           hipStream_t st) {
    AvArgs<T> a = av_args<T>(m);
    a.U = static_cast<const T *>(U);
    a.eps_out = static_cast<T *>(eps);
    a.vmax = vmax;
    return with_order(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        if (vmax)
            hipLaunchKernelGGL((k_sensor<T, P, true>), dim3(nblocks<P>(m.K)), dim3(kBlock), 0, st, a);
        else
            hipLaunchKernelGGL((k_sensor_elem<T, P>), dim3((m.K + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                               a);
        return hipGetLastError();
    });
}

hipError_t launch_sensor(const DevMesh &m, const void *U, void *eps, hipStream_t st) {
    return m.fp32 ? sensor_t<float>(m, U, eps, nullptr, st) : sensor_t<double>(m, U, eps, nullptr, st);
}

hipError_t launch_sensor_cfl(const DevMesh &m, const void *U, void *eps, unsigned long long *vmax,
                             hipStream_t st) {
    if (!m.fp32) return hipErrorInvalidValue;
    return sensor_t<float>(m, U, eps, vmax, st);
}

size_t av_args_bytes() { return sizeof(AvArgs<float>); }

void av_fill_args(const DevMesh &m, const void *U, void *eps, void *Q, unsigned long long *vmax, void *out) {
    AvArgs<float> a = av_args<float>(m);
    a.U = static_cast<const float *>(U);
    a.eps_out = static_cast<float *>(eps);
    a.eps_in = static_cast<const float *>(eps);
    a.Q = static_cast<float *>(Q);
    a.vmax = vmax;
    std::memcpy(out, &a, sizeof(a));
}

int sensor_elem_blocks(const DevMesh &m) { return (m.K + kBlock - 1) / kBlock; }

int av_tiles(const DevMesh &m) { return nblocks_rt(m.K, m.P); }

hipError_t launch_av_batch(int P, bool cfl, const void *jobs, const void *items, const int *nitems_dev,
                           int capacity, const void *eitems, const int *neitems_dev, int ecapacity,
                           hipStream_t st) {
    if (capacity <= 0) return hipSuccess;
    const auto *j = static_cast<const AvArgs<float> *>(jobs);
    const auto *it = static_cast<const int2 *>(items);
    const auto *eit = static_cast<const int2 *>(eitems);
    return with_order(P, [&](auto PC) {
        constexpr int PP = decltype(PC)::value;
        if (cfl)
            hipLaunchKernelGGL((k_sensor_batch<PP, true>), dim3(capacity), dim3(kBlock), 0, st, j, it, nitems_dev);
        else if (ecapacity > 0)
            hipLaunchKernelGGL((k_sensor_elem_batch<PP>), dim3(ecapacity), dim3(kBlock), 0, st, j, eit,
                               neitems_dev);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_avgrad_batch<PP>), dim3(capacity), dim3(kBlock), 0, st, j, it, nitems_dev);
        return hipGetLastError();
    });
}

template <typename T>
static hipError_t avgrad_t(const DevMesh &m, const void *U, const void *eps, void *Q, hipStream_t st) {
    AvArgs<T> a = av_args<T>(m);
    a.U = static_cast<const T *>(U);
    a.eps_in = static_cast<const T *>(eps);
    a.Q = static_cast<T *>(Q);
    return with_order(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_avgrad<T, P>), dim3(nblocks<P>(m.K)), dim3(kBlock), 0, st, a);
        return hipGetLastError();
    });
}

hipError_t launch_avgrad(const DevMesh &m, const void *U, const void *eps, void *Q, hipStream_t st) {
    return m.fp32 ? avgrad_t<float>(m, U, eps, Q, st) : avgrad_t<double>(m, U, eps, Q, st);
}

template <typename T>
static hipError_t cfl_t(const DevMesh &m, const void *U, const void *eps, double dt_fixed,
                        hipStream_t st) {
    hipError_t e = with_order(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        if (m.av)
            hipLaunchKernelGGL((k_cfl<T, P, true>), dim3(nblocks<P>(m.K)), dim3(kBlock), 0, st, m.K,
                               m.gamma, static_cast<const T *>(U), static_cast<const T *>(eps),
                               m.fgeo64, m.partial, m.flag);
        else
            hipLaunchKernelGGL((k_cfl<T, P, false>), dim3(nblocks<P>(m.K)), dim3(kBlock), 0, st, m.K,
                               m.gamma, static_cast<const T *>(U), static_cast<const T *>(eps),
                               m.fgeo64, m.partial, m.flag);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cfl_finish, dim3(1), dim3(kBlock), 0, st, nblocks_rt(m.K, m.P), m.partial,
                       m.cfl, dt_fixed, m.scal);
    return hipGetLastError();
}

hipError_t launch_cfl_vmax(const DevMesh &m, const void *U, unsigned long long *slot, hipStream_t st) {
    if (m.fp32) return launch_cfl_vmax_mfma(m, U, slot, st);
    hipError_t e = with_order(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        if (m.fp32)
            hipLaunchKernelGGL((k_cfl<float, P, false>), dim3(nblocks<P>(m.K)), dim3(kBlock), 0, st, m.K,
                               m.gamma, static_cast<const float *>(U), (const float *)nullptr, m.fgeo64,
                               m.partial, m.flag);
        else
            hipLaunchKernelGGL((k_cfl<double, P, false>), dim3(nblocks<P>(m.K)), dim3(kBlock), 0, st, m.K,
                               m.gamma, static_cast<const double *>(U), (const double *)nullptr, m.fgeo64,
                               m.partial, m.flag);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cfl_finish_vmax, dim3(1), dim3(kBlock), 0, st, nblocks_rt(m.K, m.P), m.partial, slot);
    return hipGetLastError();
}

hipError_t launch_cfl(const DevMesh &m, const void *U, const void *eps, double dt_fixed, hipStream_t st) {
    return m.fp32 ? cfl_t<float>(m, U, eps, dt_fixed, st) : cfl_t<double>(m, U, eps, dt_fixed, st);
}

template <typename T>
static hipError_t totals_t(const DevMesh &m, const void *U, hipStream_t st) {
    hipError_t e = with_order(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_totals<T, P>), dim3(nblocks<P>(m.K)), dim3(kBlock), 0, st, m.K,
                           static_cast<const T *>(U), m.wmass, m.partial);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finish4<SumOp>, dim3(1), dim3(kBlock), 0, st, nblocks_rt(m.K, m.P), m.partial,
                       m.scal + S_TOT, SumOp());
    return hipGetLastError();
}

hipError_t launch_totals(const DevMesh &m, const void *U, hipStream_t st) {
    return m.fp32 ? totals_t<float>(m, U, st) : totals_t<double>(m, U, st);
}

template <typename T>
static hipError_t residual_t(const DevMesh &m, const void *X, hipStream_t st) {
    hipError_t e = with_order(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_absmax<T, P>), dim3(nblocks<P>(m.K)), dim3(kBlock), 0, st, m.K,
                           static_cast<const T *>(X), m.partial);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finish4<MaxOp>, dim3(1), dim3(kBlock), 0, st, nblocks_rt(m.K, m.P), m.partial,
                       m.scal + S_RES, MaxOp());
    return hipGetLastError();
}

hipError_t launch_residual(const DevMesh &m, const void *rhs, hipStream_t st) {
    return m.fp32 ? residual_t<float>(m, rhs, st) : residual_t<double>(m, rhs, st);
}

// Prolongation of a state of order P to order Q > P (p-refinement): the
// degree-P polynomial of each element and field evaluated at the order-Q
// nodes, U_Q = I U_P with I = V_Q[:, :Np(P)] V_P^{-1} (the hierarchical modes
// of degree <= P are the first Np(P) of order Q's basis, so this is the
// paper's zero padding of the modal coefficients).  One thread per output
// value; the operator travels in the kernel arguments; sums in FP64.
struct ProlongOp {
    int np_from, np_to;
    double I[kProlongMax];
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(long n, ProlongOp op, const T *__restrict__ Uf,
                                                    T *__restrict__ Ut) {
    const long idx = (long)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= n) return;
    const long row = idx / op.np_to;          // element * 4 + field
    const int i = int(idx - row * op.np_to);
    const T *src = Uf + row * op.np_from;
    double acc = 0.0;
    for (int j = 0; j < op.np_from; ++j) acc += op.I[i * op.np_from + j] * double(src[j]);
    Ut[idx] = T(acc);
}

hipError_t launch_prolong(int K, int np_from, int np_to, const double *I, bool fp32, const void *Uf, void *Ut,
                          hipStream_t st) {
    if (np_from * np_to > kProlongMax) return hipErrorInvalidValue;
    ProlongOp op;
    op.np_from = np_from;
    op.np_to = np_to;
    for (int z = 0; z < np_from * np_to; ++z) op.I[z] = I[z];
    const long n = long(K) * kFields * np_to;
    const dim3 grid(unsigned((n + kBlock - 1) / kBlock)), block(kBlock);
    if (fp32)
        hipLaunchKernelGGL((k_prolong<float>), grid, block, 0, st, n, op, static_cast<const float *>(Uf),
                           static_cast<float *>(Ut));
    else
        hipLaunchKernelGGL((k_prolong<double>), grid, block, 0, st, n, op, static_cast<const double *>(Uf),
                           static_cast<double *>(Ut));
    return hipGetLastError();
}

hipError_t launch_eps_to_double(const DevMesh &m, const void *eps, double *out, hipStream_t st) {
    const int n = m.K;
    if (m.fp32)
        hipLaunchKernelGGL((k_eps_to_double<float>), dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0,
                           st, static_cast<const float *>(eps), out, n);
    else
        hipLaunchKernelGGL((k_eps_to_double<double>), dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0,
                           st, static_cast<const double *>(eps), out, n);
    return hipGetLastError();
}

hipError_t launch_reset_scalars(const DevMesh &m, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_scalars, dim3(1), dim3(64), 0, st, m.scal);
    return hipGetLastError();
}

}  // namespace dg
