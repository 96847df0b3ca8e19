// FP64 stage kernel on the matrix cores (v_mfma_f64_16x16x4f64) for handles
// whose elements are all straight and carry no artificial viscosity.
//
// With constant metric terms the volume term folds into the fluxes,
//   -(r_x Dr F + s_x Ds F + r_y Dr G + s_y Ds G) = -Dr F' - Ds G',
//   F' = r_x F + r_y G,  G' = s_x F + s_y G,
// and a field's right-hand side is the product
//   [LIFT  -Dr  -Ds] . [Fscale (n.F(U-) - F*); F'; G'],
// formed for column groups of 4 elements x 4 fields in three passes (face
// terms, then F', then G') over one small column-major B buffer in LDS; the
// A operand of each pass is read from the caches into registers.  Each
// element's geometry is one 128-byte FP64 record (k_pack_affine64): the
// metric terms at its first node and the normal and Fscale at each face's
// first node, one value for the whole element or face as the fold assumes
// (the per-node values of a straight element differ by rounding only, which
// Dr and Ds would amplify on small elements).  Boundary faces take the ghost
// states of the VALU kernel, and either numerical flux.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace dg {
namespace {

typedef double f64x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));

template <int P>
struct Tri64 {
    static constexpr int Np = (P + 1) * (P + 2) / 2;
    static constexpr int Nfp = P + 1;
    static constexpr int NF3 = 3 * Nfp;
    static constexpr int KSD = (Np + 3) / 4;      // k-steps of one direction
    static constexpr int KSL = (NF3 + 3) / 4;     // k-steps of the face pass
    static constexpr int KB = 4 * KSD > 4 * KSL ? 4 * KSD : 4 * KSL;
    static constexpr int KPP = KB % 8 == 4 ? KB : KB + 4;   // column stride (words / 2)
    static constexpr int MT = (Np + 15) / 16;
    static constexpr int NZ = (KSD > KSL ? KSD : KSL) * MT;
    static constexpr int NG = (NZ + 3) / 4;       // A fragments per lane per pass, in groups of 4
    static constexpr int W = 4;
    static constexpr int NTH = 64 * W;
    static constexpr int NT = W;                  // column groups per block, one per wavefront
    static constexpr int EB = 4 * NT;             // elements per block
    static constexpr int TPT = (EB * NF3 + NTH - 1) / NTH;   // face-node tasks per thread
    static constexpr int PPT = (EB * Np + NTH - 1) / NTH;    // pointwise tasks per thread
    static constexpr int NV = (EB * kFields * Np / 2 + NTH - 1) / NTH;   // 16-byte vectors per thread
    static_assert(16 * Np <= 16 * KPP, "a group's result fits in its B block");
};

struct Stage64Args {
    int K, stage, mode, riemann;
    double g, ra, rb;
    FarField<double> ff;
    const double *__restrict__ Uin;
    double *__restrict__ Uout;
    double *__restrict__ R;
    double *__restrict__ rhs;
    const int *__restrict__ nbr;       // [K][3]
    const int *__restrict__ finfo;     // [K] packed neighbour face and bc codes
    const double *__restrict__ rec;    // [K][16] r_x s_x r_y s_y | (n_x n_y Fscale) x 3 | 0 0 0
    const f64x4_t *__restrict__ opsA;  // [3][NG][64]: LIFT, -Dr, -Ds fragments; lane l of
                                       // fragment z = ks MT + mt: slot z % 4 of group z / 4
    const double *__restrict__ dt;
    // the last stage of a step in a run: also the next step's time-step
    // bound from the new state (as k_cfl: FP64 per face node with the
    // per-face-node Fscale, the state check at every node) into the slots
    int bound;
    const double *__restrict__ fgeo;   // [K][3][3 Nfp] n_x, n_y, Fscale
    unsigned long long *__restrict__ vmax;
    int *__restrict__ flag;
};

// five waves per SIMD (at most 96 registers): 901 us on the 1M-element
// P = 5 mesh, against 1,003 us at the four the default register budget gives
// and 1,151 us at six (which spills)
template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_stage_mfma64(Stage64Args a) {
    using S = Tri64<P>;
    constexpr int Np = S::Np, Nfp = S::Nfp, NF3 = S::NF3, KSD = S::KSD, KSL = S::KSL, KPP = S::KPP;
    constexpr int MT = S::MT, NG = S::NG, W = S::W, NTH = S::NTH, NT = S::NT, EB = S::EB;
    constexpr int TPT = S::TPT, PPT = S::PPT, NV = S::NV;
    __shared__ __attribute__((aligned(16))) double sB[NT][16][KPP];
    __shared__ __attribute__((aligned(16))) double sU[EB * kFields * Np];
    const long k0 = (long)blockIdx.x * EB;
    const int nel = (int)min((long)EB, (long)a.K - k0);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long base = k0 * kFields * Np;   // even: EB is a multiple of 16
    const int nflt = nel * kFields * Np;
    const int nv = nflt / 2;
    const int ntask = nel * NF3;

    // ---- loads: the tile, then the neighbour traces of this thread's
    // face-node tasks (task = element * 3 Nfp + face node; a boundary task
    // reads its own element and ignores it)
    const f64x2_t *Uv = reinterpret_cast<const f64x2_t *>(a.Uin + base);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int z = tid + v * NTH;
        if (z < nv) reinterpret_cast<f64x2_t *>(sU)[z] = Uv[z];
    }
    for (int z = 2 * nv + tid; z < nflt; z += NTH) sU[z] = a.Uin[base + z];
    int infov[TPT];
    double upn[TPT][kFields];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int task = min(tid + t * NTH, ntask - 1);
        const int e = task / NF3, q = task - e * NF3, f = q / Nfp, j = q - f * Nfp;
        const long k = k0 + e;
        infov[t] = a.finfo[k];
        const bool inner = face_bc(infov[t], f) == BC_INTERIOR;
        const long kn = inner ? (long)a.nbr[k * 3 + f] : k;
        const int vp = face_node(P, face_nbr_face(infov[t], f), Nfp - 1 - j);
#pragma unroll
        for (int c = 0; c < kFields; ++c) upn[t][c] = a.Uin[(kn * kFields + c) * Np + vp];
    }
    __syncthreads();

    f64x4_t acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    f64x4_t ga[NG];
    // one pass of the product over the wavefront's column group: B rows
    // [0, 4 KSN) against the pass's A fragments
    auto product = [&](auto KSC) {
        constexpr int KSN = decltype(KSC)::value;
        const int t = wave;
        if (4 * t < nel) {
#pragma unroll
            for (int ks = 0; ks < KSN; ++ks) {
                const double b = sB[t][lane & 15][4 * ks + (lane >> 4)];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int z = ks * MT + mt;
                    acc[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[z / 4][z % 4], b, acc[mt], 0, 0, 0);
                }
            }
        }
    };

    // ---- face terms: rows q < 3 Nfp (rows 3 Nfp .. 4 KSL zero)
    if constexpr (4 * KSL > NF3) {
        constexpr int PADR = 4 * KSL - NF3, PADN = 16 * PADR;
        for (int z = tid; z < NT * PADN; z += NTH) {
            const int t = z / PADN, rem = z - t * PADN;
            sB[t][rem / PADR][NF3 + rem % PADR] = 0.0;
        }
    }
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int task = tid + t * NTH;
        if (task < ntask) {
            const int e = task / NF3, q = task - e * NF3, f = q / Nfp, j = q - f * Nfp;
            const long k = k0 + e;
            const int vm = face_node(P, f, j);
            double um[kFields], up[kFields], d[kFields];
#pragma unroll
            for (int c = 0; c < kFields; ++c) um[c] = sU[(e * kFields + c) * Np + vm];
            const double *rc = a.rec + k * 16 + 4 + 3 * f;
            const double nx = rc[0], ny = rc[1], fs = rc[2];
            const int code = face_bc(infov[t], f);
            if (code == BC_INTERIOR) {
#pragma unroll
                for (int c = 0; c < kFields; ++c) up[c] = upn[t][c];
            } else {
                ghost_state(a.g, code, um, nx, ny, a.ff, up);
            }
            flux_jump(a.riemann, a.g, um, up, nx, ny, d);
            double(*B)[KPP] = sB[e / 4];
            const int col = (e % 4) * kFields;
#pragma unroll
            for (int c = 0; c < kFields; ++c) B[col + c][q] = fs * d[c];
        }
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) ga[g] = a.opsA[g * 64 + lane];
    // the pointwise fluxes of this thread's nodes, kept for both directions
    double Fv[PPT][kFields], Gv[PPT][kFields];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int z = min(tid + p * NTH, nel * Np - 1);
        const int el = z / Np, i = z - el * Np;
        double u[kFields];
#pragma unroll
        for (int c = 0; c < kFields; ++c) u[c] = sU[(el * kFields + c) * Np + i];
        const double ir = rcp(u[0]);
        const double vx = u[1] * ir, vy = u[2] * ir;
        const double pr = pressure_ir(a.g, u, ir);
        Fv[p][0] = u[1];
        Fv[p][1] = u[1] * vx + pr;
        Fv[p][2] = u[2] * vx;
        Fv[p][3] = (u[3] + pr) * vx;
        Gv[p][0] = u[2];
        Gv[p][1] = u[1] * vy;
        Gv[p][2] = u[2] * vy + pr;
        Gv[p][3] = (u[3] + pr) * vy;
    }
    __syncthreads();
    product(std::integral_constant<int, KSL>());

    // ---- the two directions: F' = r_x F + r_y G, then G' = s_x F + s_y G,
    // in rows i < Np (rows Np .. 4 KSD zero)
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        __syncthreads();
        if constexpr (4 * KSD > Np) {
            constexpr int PADR = 4 * KSD - Np, PADN = 16 * PADR;
            for (int z = tid; z < NT * PADN; z += NTH) {
                const int t = z / PADN, rem = z - t * PADN;
                sB[t][rem / PADR][Np + rem % PADR] = 0.0;
            }
        }
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int z = tid + p * NTH;
            if (z < nel * Np) {
                const int el = z / Np, i = z - el * Np;
                const long k = k0 + el;
                // r_x, r_y for F'; s_x, s_y for G'
                const double mf = a.rec[k * 16 + dir], mg = a.rec[k * 16 + 2 + dir];
                double(*B)[KPP] = sB[el / 4];
                const int col = (el % 4) * kFields;
#pragma unroll
                for (int c = 0; c < kFields; ++c) B[col + c][i] = mf * Fv[p][c] + mg * Gv[p][c];
            }
        }
#pragma unroll
        for (int g = 0; g < NG; ++g) ga[g] = a.opsA[((1 + dir) * NG + g) * 64 + lane];
        __syncthreads();
        product(std::integral_constant<int, KSD>());
    }
    __syncthreads();
    // the result over the wavefront's own B block as [element % 4][field][node]
    // (accumulator slot r of lane l is row 16 mt + l / 16 + 4 r, column l % 16)
    {
        const int t = wave;
        const int col = lane & 15, le = col / kFields, c = col - le * kFields;
        if (4 * t + le < nel) {
            double *res = &sB[t][0][0];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 16 * mt + (lane >> 4) + 4 * r;
                    if (i < Np) res[(le * kFields + c) * Np + i] = acc[mt][r];
                }
        }
    }
    __syncthreads();

    // ---- epilogue: Runge-Kutta update (or the bare rhs) in 16-byte vectors
    const double dt = a.mode ? *a.dt : 0.0;
    const bool rk_read = a.mode && a.stage > 0;
    auto result = [&](int z) -> double {
        const int el = z / (kFields * Np), off = z - el * (kFields * Np);
        return (&sB[el / 4][0][0])[(el % 4) * kFields * Np + off];
    };
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int zv = tid + v * NTH;
        if (zv < nv) {
            const f64x2_t rh = {result(2 * zv), result(2 * zv + 1)};
            if (a.mode == 0) {
                reinterpret_cast<f64x2_t *>(a.rhs + base)[zv] = rh;
            } else {
                const f64x2_t rold = rk_read ? reinterpret_cast<const f64x2_t *>(a.R + base)[zv] : f64x2_t{0.0, 0.0};
                const f64x2_t rr = a.stage == 0 ? dt * rh : a.ra * rold + dt * rh;
                const f64x2_t un = reinterpret_cast<const f64x2_t *>(sU)[zv] + a.rb * rr;
                reinterpret_cast<f64x2_t *>(a.R + base)[zv] = rr;
                reinterpret_cast<f64x2_t *>(a.Uout + base)[zv] = un;
                if (a.bound) reinterpret_cast<f64x2_t *>(sU)[zv] = un;
            }
        }
    }
    for (int z = 2 * nv + tid; z < nflt; z += NTH) {
        const double rh = result(z);
        const long idx = base + z;
        if (a.mode == 0) {
            a.rhs[idx] = rh;
        } else {
            const double rr = a.stage == 0 ? dt * rh : a.ra * a.R[idx] + dt * rh;
            const double un = sU[z] + a.rb * rr;
            a.R[idx] = rr;
            a.Uout[idx] = un;
            if (a.bound) sU[z] = un;
        }
    }
    if (a.bound) {
        __shared__ double sRed[W];
        __syncthreads();
        int bad = 0;
        for (int z = tid; z < nel * Np; z += NTH) {
            const int el = z / Np, i = z - el * Np;
            double u[kFields];
#pragma unroll
            for (int c = 0; c < kFields; ++c) u[c] = sU[(el * kFields + c) * Np + i];
            if (bad_state(a.g, u)) bad = 1;
        }
        double best = 0.0;
        for (int z = tid; z < ntask; z += NTH) {
            const int e = z / NF3, q = z - e * NF3, f = q / Nfp, j = q - f * Nfp;
            const int v = face_node(P, f, j);
            double u[kFields];
#pragma unroll
            for (int c = 0; c < kFields; ++c) u[c] = sU[(e * kFields + c) * Np + v];
            const double b = cfl_bound(a.g, u, a.fgeo[((k0 + e) * 3 + 2) * NF3 + q], 0.0, P + 1.0);
            best = b > best ? b : best;
        }
        if (__any(bad) && lane == 0) atomicOr(a.flag, 1);
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(best, off);
            best = o > best ? o : best;
        }
        if (lane == 0) sRed[wave] = best;
        __syncthreads();
        if (tid == 0) {
            double m = sRed[0];
            for (int w = 1; w < W; ++w) m = sRed[w] > m ? sRed[w] : m;
            atomicMax(a.vmax + (blockIdx.x & (kVmaxSlots - 1)), (unsigned long long)__double_as_longlong(m));
        }
    }
}

// dt = CFL / bound from the slots (or the fixed step), booked into the
// scalars as k_cfl_finish does; clears the slots.  One wavefront of
// kVmaxSlots lanes.
__global__ void k_dt_slots64(double cfl, double dt_fixed, unsigned long long *__restrict__ slots,
                             double *__restrict__ scal) {
    const int l = threadIdx.x;
    unsigned long long v = slots[l];
    for (int off = kVmaxSlots / 2; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    slots[l] = 0ull;
    if (l != 0) return;
    const double vmax = __longlong_as_double((long long)v);
    const double dt = dt_fixed > 0.0 ? dt_fixed : cfl * (1.0 / vmax);
    scal[S_DT] = dt;
    scal[S_T] += dt;
    scal[S_DTMIN] = dt < scal[S_DTMIN] ? dt : scal[S_DTMIN];
    scal[S_DTMAX] = dt > scal[S_DTMAX] ? dt : scal[S_DTMAX];
    scal[S_STEPS] += 1.0;
}

// The 128-byte geometry record of each (straight) element.
__global__ void k_pack_affine64(int K, int Np, int Nfp, const double *__restrict__ geo,
                                const double *__restrict__ fgeo, double *__restrict__ rec) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int NF3 = 3 * Nfp;
    double *r = rec + k * 16;
    for (int m = 0; m < 4; ++m) r[m] = geo[(k * 4 + m) * Np];
    for (int f = 0; f < 3; ++f)
        for (int m = 0; m < 3; ++m) r[4 + 3 * f + m] = fgeo[(k * 3 + m) * NF3 + f * Nfp];
    r[13] = r[14] = r[15] = 0.0;
}

template <typename F>
auto with_order64(int P, F &&f) {
    switch (P) {
        case 1: return f(std::integral_constant<int, 1>());
        case 2: return f(std::integral_constant<int, 2>());
        case 3: return f(std::integral_constant<int, 3>());
        case 4: return f(std::integral_constant<int, 4>());
        default: return f(std::integral_constant<int, 5>());
    }
}

}  // namespace

size_t mfma64_opsA_values(int P) {
    return with_order64(P, [](auto PC) { return size_t(3) * Tri64<decltype(PC)::value>::NG * 64 * 4; });
}

void mfma64_fill_opsA(int P, const double *Dr, const double *Ds, const double *LIFT, double *out) {
    with_order64(P, [&](auto PC) {
        using S = Tri64<decltype(PC)::value>;
        constexpr int Np = S::Np, NF3 = S::NF3, MT = S::MT, NG = S::NG;
        std::fill(out, out + size_t(3) * NG * 64 * 4, 0.0);
        for (int pass = 0; pass < 3; ++pass) {
            const int ksn = pass == 0 ? S::KSL : S::KSD;
            for (int mt = 0; mt < MT; ++mt)
                for (int l = 0; l < 64; ++l)
                    for (int ks = 0; ks < ksn; ++ks) {
                        const int m = 16 * mt + (l & 15), k = 4 * ks + (l >> 4);
                        double v = 0.0;
                        if (m < Np) {
                            if (pass == 0)
                                v = k < NF3 ? LIFT[m * NF3 + k] : 0.0;
                            else if (k < Np)
                                v = -(pass == 1 ? Dr : Ds)[m * Np + k];
                        }
                        const int z = ks * MT + mt;
                        out[((size_t(pass) * NG + z / 4) * 64 + l) * 4 + z % 4] = v;
                    }
        }
        return 0;
    });
}

hipError_t launch_pack_affine64(const DevMesh &m, double *rec, hipStream_t st) {
    hipLaunchKernelGGL(k_pack_affine64, dim3((m.K + 127) / 128), dim3(128), 0, st, m.K, m.Np, m.Nfp, m.geo64,
                       m.fgeo64, rec);
    return hipGetLastError();
}

hipError_t launch_dt_slots64(const DevMesh &m, double dt_fixed, hipStream_t st) {
    hipLaunchKernelGGL(k_dt_slots64, dim3(1), dim3(kVmaxSlots), 0, st, m.cfl, dt_fixed, m.vmax, m.scal);
    return hipGetLastError();
}

hipError_t launch_stage_mfma64(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                               bool bound, hipStream_t st) {
    Stage64Args a;
    a.K = m.K;
    a.stage = stage;
    a.mode = rhs ? 0 : 1;
    a.riemann = m.riemann;
    a.g = m.gamma;
    a.ra = rk_a(stage);
    a.rb = rk_b(stage);
    a.ff = make_farfield<double>(m.gamma, m.qinf);
    a.Uin = static_cast<const double *>(Uin);
    a.Uout = static_cast<double *>(Uout);
    a.R = static_cast<double *>(R);
    a.rhs = static_cast<double *>(rhs);
    a.nbr = m.nbr;
    a.finfo = m.finfo;
    a.rec = m.geoA64;
    a.opsA = reinterpret_cast<const f64x4_t *>(m.opsA64);
    a.dt = m.scal + S_DT;
    a.bound = bound && !rhs && m.vmax ? 1 : 0;
    a.fgeo = m.fgeo64;
    a.vmax = m.vmax;
    a.flag = m.flag;
    return with_order64(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        using S = Tri64<P>;
        const int blocks = (m.K + S::EB - 1) / S::EB;
        hipLaunchKernelGGL((k_stage_mfma64<P>), dim3(blocks), dim3(S::NTH), 0, st, a);
        return hipGetLastError();
    });
}

}  // namespace dg
