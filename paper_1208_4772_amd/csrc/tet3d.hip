// 3D nodal DG on straight tetrahedra, five fields (rho, rho u, rho v, rho w,
// E): the paper's own setting (Section 2; the 3D Euler system of Section 5).
//
//   dU/dt = -(r_x Dr + s_x Ds + t_x Dt) F - (r_y ...) G - (r_z ...) H
//           + LIFT (Fscale (n.F(U-) - F*)),   F* local Lax-Friedrichs
//
// on a reference tetrahedron with vertices (-1,-1,-1), (1,-1,-1), (-1,1,-1),
// (-1,-1,1), faces (v1 v2 v3), (v1 v2 v4), (v2 v3 v4), (v1 v3 v4), and
// equispaced nodes (the lattice (i, j, k)/P, r fastest).  A straight element
// has constant metric terms, normals and Fscale per face: 25 numbers.
//
// The stage runs on the matrix cores in both precisions (k_stage3_mfma,
// FP32; k_stage3_mfma64, FP64): with constant metric terms the volume term
// folds into contravariant fluxes, F_a = sum_d (d r_a / d x_d) F_d, and the
// whole right-hand side of a field is one product
//   rhs = [-Dr  -Ds  -Dt  LIFT] (Np x (3 Np + 4 Nfp)) . [F_r; F_s; F_t; Fscale (n.F - F*)],
// formed for column groups of 3 elements x 5 fields (15 of 16 columns) with
// v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64, in four passes (faces, then
// r, s, t) that share one B buffer in LDS; the A operand of each pass (the
// same for every block) is read from the caches into registers.  Face
// terms: one thread per face node, the neighbour's trace gathered through a
// precomputed node map, the mirror state at walls.  The time step is
// reduced in FP64 from the state (k_cfl3, k_dt3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace dg {
namespace {

constexpr int kF3 = 5;          // fields
constexpr int kB3 = 256;        // threads per block
constexpr int kGeo3 = 25;       // r_x r_y r_z s_x s_y s_z t_x t_y t_z | (n_x n_y n_z) x 4 | Fscale x 4

// Elements per block of the time-step bound kernel: about two face-node
// tasks per thread.
template <int P>
struct Bound3 {
    static constexpr int Nfp = (P + 1) * (P + 2) / 2;
    static constexpr int NF4 = 4 * Nfp;
    static constexpr int EB = 2 * kB3 / NF4;
};

template <typename T>
__device__ inline void euler3_flux(T g, const T u[kF3], T F[kF3], T G[kF3], T H[kF3]) {
    const T ir = rcp(u[0]);
    const T vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
    const T p = (g - T(1)) * (u[4] - T(0.5) * (u[1] * vx + u[2] * vy + u[3] * vz));
    F[0] = u[1]; F[1] = u[1] * vx + p; F[2] = u[2] * vx; F[3] = u[3] * vx; F[4] = (u[4] + p) * vx;
    G[0] = u[2]; G[1] = u[1] * vy; G[2] = u[2] * vy + p; G[3] = u[3] * vy; G[4] = (u[4] + p) * vy;
    H[0] = u[3]; H[1] = u[1] * vz; H[2] = u[2] * vz; H[3] = u[3] * vz + p; H[4] = (u[4] + p) * vz;
}

// n.F(u) and |v.n| + c
template <typename T>
__device__ inline void normal_flux3(T g, const T u[kF3], T nx, T ny, T nz, T fn[kF3], T &lam) {
    const T ir = rcp(u[0]);
    const T vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
    const T p = (g - T(1)) * (u[4] - T(0.5) * (u[1] * vx + u[2] * vy + u[3] * vz));
    const T vn = vx * nx + vy * ny + vz * nz;
    fn[0] = u[0] * vn;
    fn[1] = u[1] * vn + p * nx;
    fn[2] = u[2] * vn + p * ny;
    fn[3] = u[3] * vn + p * nz;
    fn[4] = (u[4] + p) * vn;
    lam = fabs(vn) + fsqrt(g * p * ir);
}

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));

// Vector types of the matrix-core stage per precision: V4, an accumulator
// (and a group of four A fragments); V16, one 16-byte access (VW values).
template <typename T>
struct VT;
template <>
struct VT<float> {
    typedef f32x4_t V4;
    typedef f32x4_t V16;
    static constexpr int VW = 4;
};
template <>
struct VT<double> {
    typedef f64x4_t V4;
    typedef f64x2_t V16;
    static constexpr int VW = 2;
};
__device__ __forceinline__ f32x4_t mfma16(float a, float b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4_t mfma16(double a, double b, f64x4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Shape of the matrix-core stage, in four passes over one small B buffer:
// the face terms (LIFT, 4 Nfp rows), then the contravariant fluxes along
// r, s and t (Dr, Ds, Dt, Np rows each, padded to whole k-steps).  Small
// LDS per element keeps several blocks on a CU to hide memory latency (at
// P = 4: 25 KB and 91 registers, five blocks per CU; one pass over a
// 3 Np + 4 Nfp row buffer took 53 KB and 166 registers, three blocks, and
// 33% more time).  The B operand is stored column-major with a column
// stride KPP = 4 (mod 8) words: the flux writes (consecutive rows) and the
// fragment reads (16 columns x 4 rows) then spread over the LDS banks.
template <int P>
struct TetM {
    static constexpr int Np = (P + 1) * (P + 2) * (P + 3) / 6;
    static constexpr int Nfp = (P + 1) * (P + 2) / 2;
    static constexpr int NF4 = 4 * Nfp;
    static constexpr int KSD = (Np + 3) / 4;       // k-steps of one direction
    static constexpr int KSL = NF4 / 4;            // k-steps of the face pass
    static constexpr int KB = 4 * KSD > NF4 ? 4 * KSD : NF4;
    static constexpr int KPP = KB % 8 == 4 ? KB : KB + 4;
    static constexpr int MT = (Np + 15) / 16;
    static constexpr int NZD = KSD * MT, NGD = (NZD + 3) / 4;
    static constexpr int NZL = KSL * MT, NGL = (NZL + 3) / 4;
    static constexpr int W = 4;
    static constexpr int NTH = 64 * W;
    // one column group per wavefront: measured on 26,112 tetrahedra, 8, 12
    // or 16 groups per block are 8-100% slower at every order (fewer blocks
    // per CU to hide the memory latency)
    static constexpr int NT = W;
    static constexpr int GW = NT / W;              // column groups per wavefront
    static constexpr int EB = 3 * NT;
    static constexpr int TPT = (EB * NF4 + NTH - 1) / NTH;   // face-node tasks per thread
    static constexpr int PPT = (EB * Np + NTH - 1) / NTH;    // pointwise tasks per thread
    static_assert(NF4 % 4 == 0, "face rows are whole k-steps");
    static_assert(15 * Np <= 16 * KPP, "a group's result fits in its B block");
};

template <typename T>
struct Stage3MArgs {
    int K, stage, mode;
    T g, ra, rb;
    const T *__restrict__ Uin;
    T *__restrict__ Uout;
    T *__restrict__ R;
    T *__restrict__ rhs;
    const T *__restrict__ geo;
    const int *__restrict__ fmap;
    const int *__restrict__ fmask;
    const typename VT<T>::V4 *__restrict__ opsA;  // [4][NG][64]: face, then r, s, t fragments (NG = max(NGL, NGD));
                                                  // lane l of fragment z = ks MT + mt: slot z % 4 of group z / 4
    const double *__restrict__ dt;
    // the last stage of a step: also the time-step bound of the new state
    // (as k_cfl3) into the slots, and its state check
    int bound;
    double gamma;
    unsigned long long *__restrict__ vmax;
    int *__restrict__ flag;
};

// The stage body for FP32 (k_stage3_mfma) and FP64 (k_stage3_mfma64).  FP32
// keeps each node's pointwise fluxes in registers across the three direction
// passes and requests the Runge-Kutta register before the product; FP64
// (twice the registers per value) recomputes the fluxes per pass and reads
// the register in the epilogue.
template <typename T, int P>
__device__ __forceinline__ void stage3_mfma_body(const Stage3MArgs<T> &a) {
    using S = TetM<P>;
    using V4 = typename VT<T>::V4;
    using V16 = typename VT<T>::V16;
    constexpr int VW = VT<T>::VW;
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int Np = S::Np, NF4 = S::NF4, KSD = S::KSD, KSL = S::KSL, KPP = S::KPP, MT = S::MT;
    constexpr int W = S::W, NTH = S::NTH, NT = S::NT, GW = S::GW, EB = S::EB, NGD = S::NGD, NGL = S::NGL;
    constexpr int TPT = S::TPT, PPT = S::PPT;
    constexpr int NG = NGL > NGD ? NGL : NGD;
    constexpr int NV = (EB * kF3 * Np / VW + NTH - 1) / NTH;   // 16-byte vectors of a full tile per thread
    static_assert(EB * kF3 * Np % VW == 0, "a full tile is whole 16-byte vectors");
    __shared__ __attribute__((aligned(16))) T sB[NT][16][KPP];
    __shared__ __attribute__((aligned(16))) T sU[EB * kF3 * Np];
    __shared__ T sG[EB * kGeo3];
    __shared__ int sFM[NF4];
    const long k0 = (long)blockIdx.x * EB;
    const int nel = (int)min((long)EB, (long)a.K - k0);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long base = k0 * kF3 * Np;   // 16-byte aligned: EB is a multiple of 12
    const int nflt = nel * kF3 * Np;
    const int nv = nflt / VW;           // whole vectors of this tile (the rest: scalar tail)
    const int ntask = nel * NF4;

    const V16 *Uv = reinterpret_cast<const V16 *>(a.Uin + base);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int z = tid + v * NTH;
        if (z < nv) reinterpret_cast<V16 *>(sU)[z] = Uv[z];
    }
    for (int z = VW * nv + tid; z < nflt; z += NTH) sU[z] = a.Uin[base + z];
    for (int z = tid; z < nel * kGeo3; z += NTH) sG[z] = a.geo[k0 * kGeo3 + z];
    for (int z = tid; z < NF4; z += NTH) sFM[z] = a.fmask[z];
    int nbv[TPT];
    T upn[TPT][kF3];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int task = min(tid + t * NTH, ntask - 1);
        const int e = task / NF4, q = task - e * NF4;
        nbv[t] = a.fmap[(k0 + e) * NF4 + q];
        const long src = nbv[t] >= 0 ? (long)nbv[t] : (k0 + e) * kF3 * Np;
#pragma unroll
        for (int c = 0; c < kF3; ++c) upn[t][c] = a.Uin[src + c * Np];
    }
    __syncthreads();

    V4 acc[GW][MT];
#pragma unroll
    for (int gi = 0; gi < GW; ++gi)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[gi][mt] = V4{T(0), T(0), T(0), T(0)};
    auto product = [&](const V4(&ga)[NG], auto KSC) {
        constexpr int KSN = decltype(KSC)::value;
#pragma unroll
        for (int gi = 0; gi < GW; ++gi) {
            const int t = wave + gi * W;
            if (3 * t < nel) {
#pragma unroll
                for (int ks = 0; ks < KSN; ++ks) {
                    const T b = sB[t][lane & 15][4 * ks + (lane >> 4)];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const int z = ks * MT + mt;
                        acc[gi][mt] = mfma16(ga[z / 4][z % 4], b, acc[gi][mt]);
                    }
                }
            }
        }
    };
    V4 ga[NG];

    // ---- face terms: rows q < 4 Nfp
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int task = tid + t * NTH;
        if (task < ntask) {
            const int e = task / NF4, q = task - e * NF4, f = q / (NF4 / 4);
            const int vm = sFM[q];
            const T *gm = sG + e * kGeo3;
            const T nx = gm[9 + 3 * f], ny = gm[10 + 3 * f], nz = gm[11 + 3 * f], fs = gm[21 + f];
            T um[kF3], up[kF3];
#pragma unroll
            for (int c = 0; c < kF3; ++c) um[c] = sU[(e * kF3 + c) * Np + vm];
            if (nbv[t] >= 0) {
#pragma unroll
                for (int c = 0; c < kF3; ++c) up[c] = upn[t][c];
            } else {
                const T mn = um[1] * nx + um[2] * ny + um[3] * nz;
                up[0] = um[0];
                up[1] = um[1] - T(2) * mn * nx;
                up[2] = um[2] - T(2) * mn * ny;
                up[3] = um[3] - T(2) * mn * nz;
                up[4] = um[4];
            }
            T fm[kF3], fp[kF3], lm, lp;
            normal_flux3(a.g, um, nx, ny, nz, fm, lm);
            normal_flux3(a.g, up, nx, ny, nz, fp, lp);
            const T lam = lm > lp ? lm : lp;
            T(*B)[KPP] = sB[e / 3];
            const int col = (e % 3) * kF3;
#pragma unroll
            for (int c = 0; c < kF3; ++c)
                B[col + c][q] = fs * (T(0.5) * (fm[c] - fp[c]) + T(0.5) * lam * (up[c] - um[c]));
        }
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) ga[g] = a.opsA[g * 64 + lane];
    // FP32: the pointwise fluxes of this thread's nodes, kept in registers
    // for the three direction passes
    constexpr int KP_ = F32 ? PPT : 1;
    T Fx[KP_][kF3], Fy[KP_][kF3], Fz[KP_][kF3];
    if constexpr (F32) {
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int z = min(tid + p * NTH, nel * Np - 1);
            const int el = z / Np, i = z - el * Np;
            T u[kF3];
#pragma unroll
            for (int c = 0; c < kF3; ++c) u[c] = sU[(el * kF3 + c) * Np + i];
            euler3_flux(a.g, u, Fx[p], Fy[p], Fz[p]);
        }
    }
    __syncthreads();
    product(ga, std::integral_constant<int, KSL>());

    // ---- the three directions: rows i < Np (rows Np .. 4 KSD zero)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        __syncthreads();
        if constexpr (4 * KSD > Np) {
            constexpr int PADR = 4 * KSD - Np, PADN = 16 * PADR;
            for (int z = tid; z < NT * PADN; z += NTH) {
                const int t = z / PADN, rem = z - t * PADN;
                sB[t][rem / PADR][Np + rem % PADR] = T(0);
            }
        }
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int z = tid + p * NTH;
            if (z < nel * Np) {
                const int el = z / Np, i = z - el * Np;
                const T *m = sG + el * kGeo3 + 3 * d;
                const T m0 = m[0], m1 = m[1], m2 = m[2];
                T(*B)[KPP] = sB[el / 3];
                const int col = (el % 3) * kF3;
                if constexpr (F32) {
#pragma unroll
                    for (int c = 0; c < kF3; ++c) B[col + c][i] = m0 * Fx[p][c] + m1 * Fy[p][c] + m2 * Fz[p][c];
                } else {
                    T u[kF3], F[kF3], G[kF3], H[kF3];
#pragma unroll
                    for (int c = 0; c < kF3; ++c) u[c] = sU[(el * kF3 + c) * Np + i];
                    euler3_flux(a.g, u, F, G, H);
#pragma unroll
                    for (int c = 0; c < kF3; ++c) B[col + c][i] = m0 * F[c] + m1 * G[c] + m2 * H[c];
                }
            }
        }
#pragma unroll
        for (int g = 0; g < NG; ++g) ga[g] = a.opsA[((1 + d) * NG + g) * 64 + lane];
        __syncthreads();
        product(ga, std::integral_constant<int, KSD>());
    }
    constexpr int NR = F32 ? NV : 1;
    V16 rv[NR];
    const bool rk_read = a.mode && a.stage > 0;
    if constexpr (F32) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int z = min(tid + v * NTH, nv - 1);
            rv[v] = rk_read && nv > 0 ? reinterpret_cast<const V16 *>(a.R + base)[z] : V16{};
        }
    }
    __syncthreads();
#pragma unroll
    for (int gi = 0; gi < GW; ++gi) {
        const int t = wave + gi * W;
        const int col = lane & 15, le = col / kF3, c = col - le * kF3;
        if (col < 15 && 3 * t + le < nel) {
            T *res = &sB[t][0][0];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // output row of accumulator slot r: four consecutive rows
                    // per 16-lane group in FP32, rows interleaved by 4 in FP64
                    const int i = F32 ? 16 * mt + 4 * (lane >> 4) + r : 16 * mt + (lane >> 4) + 4 * r;
                    if (i < Np) res[(le * kF3 + c) * Np + i] = acc[gi][mt][r];
                }
        }
    }
    __syncthreads();

    // ---- epilogue: Runge-Kutta update (or the bare rhs) in 16-byte vectors
    // where the tile is whole vectors
    const T dt = a.mode ? T(*a.dt) : T(0);
    auto result = [&](int z) -> T {
        const int el = z / (kF3 * Np), off = z - el * (kF3 * Np);
        return (&sB[el / 3][0][0])[(el % 3) * kF3 * Np + off];
    };
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int zv = tid + v * NTH;
        if (zv < nv) {
            V16 rh;
#pragma unroll
            for (int e = 0; e < VW; ++e) rh[e] = result(VW * zv + e);
            if (a.mode == 0) {
                reinterpret_cast<V16 *>(a.rhs + base)[zv] = rh;
            } else {
                V16 rold;
                if constexpr (F32)
                    rold = rv[v];
                else
                    rold = rk_read ? reinterpret_cast<const V16 *>(a.R + base)[zv] : V16{};
                const V16 rr = a.stage == 0 ? dt * rh : a.ra * rold + dt * rh;
                const V16 un = reinterpret_cast<const V16 *>(sU)[zv] + a.rb * rr;
                reinterpret_cast<V16 *>(a.R + base)[zv] = rr;
                reinterpret_cast<V16 *>(a.Uout + base)[zv] = un;
                if (a.bound) reinterpret_cast<V16 *>(sU)[zv] = un;
            }
        }
    }
    for (int z = VW * nv + tid; z < nflt; z += NTH) {
        const T rh = result(z);
        const long idx = base + z;
        if (a.mode == 0) {
            a.rhs[idx] = rh;
        } else {
            const T rr = a.stage == 0 ? dt * rh : a.ra * a.R[idx] + dt * rh;
            const T un = sU[z] + a.rb * rr;
            a.R[idx] = rr;
            a.Uout[idx] = un;
            if (a.bound) sU[z] = un;
        }
    }
    if (a.bound) {
        // the next step's bound from the new state, node for node as k_cfl3:
        // FP64 at every face node, maximum per block into a slot
        __shared__ double sRed[W];
        __syncthreads();
        double best = 0.0;
        int bad = 0;
        for (int z = tid; z < ntask; z += NTH) {
            const int e = z / NF4, q = z - e * NF4, f = q / (NF4 / 4);
            const int v = sFM[q];
            double u[kF3];
#pragma unroll
            for (int c = 0; c < kF3; ++c) u[c] = double(sU[(e * kF3 + c) * Np + v]);
            const double ir = 1.0 / u[0];
            const double vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
            const double p = (a.gamma - 1.0) * (u[4] - 0.5 * (u[1] * vx + u[2] * vy + u[3] * vz));
            if (!(u[0] > 0.0) || !(p > 0.0) || !isfinite(u[1]) || !isfinite(u[2]) || !isfinite(u[3]) ||
                !isfinite(u[4]) || !isfinite(p))
                bad = 1;
            const double lam = sqrt(vx * vx + vy * vy + vz * vz) + sqrt(a.gamma * p * ir);
            const double b = 0.5 * (P + 1.0) * (P + 1.0) * double(sG[e * kGeo3 + 21 + f]) * lam;
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
            atomicMax(a.vmax + (blockIdx.x & (kSlots3 - 1)), (unsigned long long)__double_as_longlong(m));
        }
    }
}

template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_stage3_mfma(Stage3MArgs<float> a) {
    stage3_mfma_body<float, P>(a);
}

template <int P>
__global__ __launch_bounds__(256) void k_stage3_mfma64(Stage3MArgs<double> a) {
    stage3_mfma_body<double, P>(a);
}

// Time-step bound in FP64 at every face node: (P+1)^2 Fscale (|v| + c) / 2,
// maximum per block into one of kSlots3 slots (block id mod kSlots3, so that
// the atomics of thousands of blocks do not queue on one address;
// non-negative doubles order like their bit patterns); the state check
// (non-finite, rho <= 0, p <= 0) at every face node.
template <typename T, int P>
__global__ __launch_bounds__(kB3) void k_cfl3(int K, double g, const T *__restrict__ U, const T *__restrict__ geo,
                                             const int *__restrict__ fmask, unsigned long long *vmax,
                                             int *flag) {
    constexpr int Np = (P + 1) * (P + 2) * (P + 3) / 6, NF4 = Bound3<P>::NF4, EB = Bound3<P>::EB;
    __shared__ double sRed[kB3 / 64];
    const long k0 = (long)blockIdx.x * EB;
    const int nel = (int)min((long)EB, (long)K - k0);
    double best = 0.0;
    int bad = 0;
    for (int z = threadIdx.x; z < nel * NF4; z += kB3) {
        const int e = z / NF4, q = z - e * NF4, f = q / (NF4 / 4);
        const long k = k0 + e;
        const int v = fmask[q];
        double u[kF3];
#pragma unroll
        for (int c = 0; c < kF3; ++c) u[c] = double(U[(k * kF3 + c) * Np + v]);
        const double ir = 1.0 / u[0];
        const double vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
        const double p = (g - 1.0) * (u[4] - 0.5 * (u[1] * vx + u[2] * vy + u[3] * vz));
        if (!(u[0] > 0.0) || !(p > 0.0) || !isfinite(u[1]) || !isfinite(u[2]) || !isfinite(u[3]) ||
            !isfinite(u[4]) || !isfinite(p))
            bad = 1;
        const double lam = sqrt(vx * vx + vy * vy + vz * vz) + sqrt(g * p * ir);
        const double fs = double(geo[k * kGeo3 + 21 + f]);
        const double b = 0.5 * (P + 1.0) * (P + 1.0) * fs * lam;
        best = b > best ? b : best;
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(best, off);
        best = o > best ? o : best;
    }
    if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sRed[0];
        for (int w = 1; w < kB3 / 64; ++w) m = sRed[w] > m ? sRed[w] : m;
        atomicMax(vmax + (blockIdx.x & (kSlots3 - 1)), (unsigned long long)__double_as_longlong(m));
    }
}

// dt = CFL / bound (or the fixed step), booked into the scalars; clears the
// slots for the next step.  One wavefront of kSlots3 lanes.
__global__ void k_dt3(double cfl, double dt_fixed, unsigned long long *vmax, double *scal) {
    const int l = threadIdx.x;
    unsigned long long v = vmax[l];
    for (int off = kSlots3 / 2; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    vmax[l] = 0ull;
    if (l != 0) return;
    const double b = __longlong_as_double((long long)v);
    const double dt = dt_fixed > 0.0 ? dt_fixed : cfl / b;
    scal[S_DT] = dt;
    scal[S_T] += dt;
    scal[S_DTMIN] = dt < scal[S_DTMIN] ? dt : scal[S_DTMIN];
    scal[S_DTMAX] = dt > scal[S_DTMAX] ? dt : scal[S_DTMAX];
    scal[S_STEPS] += 1.0;
}

// Straight-element geometry in FP64: metric terms from the vertex
// coordinates (the affine map's columns x_r = (v2 - v1)/2, ...), outward unit
// normals and Fscale = (face area / 2) / (volume / (4/3)) per face.
__global__ void k_geometry3(int K, const double *__restrict__ X, double *__restrict__ geo,
                            int *__restrict__ count) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const double *v = X + k * 12;
    double A[3][3];   // A[d][a] = d x_d / d r_a
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) A[d][c] = 0.5 * (v[3 * (c + 1) + d] - v[d]);
    const double J = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                     A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                     A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    if (!(J > 0.0)) atomicAdd(count, 1);
    double *g = geo + k * kGeo3;
    // inverse: row a of A^-1 is grad r_a
    const double iJ = 1.0 / J;
    g[0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) * iJ;
    g[1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * iJ;
    g[2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * iJ;
    g[3] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) * iJ;
    g[4] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * iJ;
    g[5] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * iJ;
    g[6] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) * iJ;
    g[7] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * iJ;
    g[8] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * iJ;
    const int fv[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};
    const int opp[4] = {3, 2, 0, 1};
    for (int f = 0; f < 4; ++f) {
        const double *pa = v + 3 * fv[f][0], *pb = v + 3 * fv[f][1], *pc = v + 3 * fv[f][2], *po = v + 3 * opp[f];
        const double e1[3] = {pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]};
        const double e2[3] = {pc[0] - pa[0], pc[1] - pa[1], pc[2] - pa[2]};
        double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const double twice_area = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        const double toward = n[0] * (po[0] - pa[0]) + n[1] * (po[1] - pa[1]) + n[2] * (po[2] - pa[2]);
        const double sgn = toward > 0.0 ? -1.0 : 1.0;
        for (int d = 0; d < 3; ++d) g[9 + 3 * f + d] = sgn * n[d] / twice_area;
        g[21 + f] = (0.25 * twice_area) / J;
    }
}

__global__ void k_reset3(double *scal, unsigned long long *vmax, int *flag) {
    const int l = threadIdx.x;
    vmax[l] = 0ull;
    if (l != 0) return;
    for (int i = 0; i < S_NSCAL; ++i) scal[i] = 0.0;
    scal[S_DTMIN] = __longlong_as_double(0x7ff0000000000000ll);   // +inf
    *flag = 0;
}

template <typename F>
auto with_order3(int P, F &&f) {
    switch (P) {
        case 1: return f(std::integral_constant<int, 1>());
        case 2: return f(std::integral_constant<int, 2>());
        case 3: return f(std::integral_constant<int, 3>());
        default: return f(std::integral_constant<int, 4>());
    }
}

}  // namespace

int tet3_blocks(int K, int P) {
    return with_order3(P, [&](auto PC) {
        constexpr int EB = Bound3<decltype(PC)::value>::EB;
        return (K + EB - 1) / EB;
    });
}

hipError_t launch_reset3(const Tet3Mesh &m, hipStream_t st) {
    hipLaunchKernelGGL(k_reset3, dim3(1), dim3(kSlots3), 0, st, m.scal, m.vmax, m.flag);
    return hipGetLastError();
}

hipError_t launch_geometry3(int K, const double *X, double *geo, int *count, hipStream_t st) {
    hipLaunchKernelGGL(k_geometry3, dim3((K + 127) / 128), dim3(128), 0, st, K, X, geo, count);
    return hipGetLastError();
}

template <int P>
constexpr int tet3_ng() {
    using S = TetM<P>;
    return S::NGL > S::NGD ? S::NGL : S::NGD;
}

size_t tet3_mfma_opsA_values(int P) {
    return with_order3(P, [](auto PC) { return size_t(4) * tet3_ng<decltype(PC)::value>() * 64 * 4; });
}

template <typename T>
static void fill_opsA3(int P, const double *Dr, const double *Ds, const double *Dt, const double *LIFT, T *out) {
    with_order3(P, [&](auto PC) {
        constexpr int PP = decltype(PC)::value;
        using S = TetM<PP>;
        constexpr int Np = S::Np, NF4 = S::NF4, MT = S::MT, NG = tet3_ng<PP>();
        std::fill(out, out + size_t(4) * NG * 64 * 4, T(0));
        const double *D[3] = {Dr, Ds, Dt};
        for (int pass = 0; pass < 4; ++pass) {
            const int ksn = pass == 0 ? S::KSL : S::KSD;
            for (int mt = 0; mt < MT; ++mt)
                for (int l = 0; l < 64; ++l)
                    for (int ks = 0; ks < ksn; ++ks) {
                        const int m = 16 * mt + (l & 15), k = 4 * ks + (l >> 4);
                        double v = 0.0;
                        if (m < Np) {
                            if (pass == 0)
                                v = LIFT[m * NF4 + k];
                            else if (k < Np)
                                v = -D[pass - 1][m * Np + k];
                        }
                        const int z = ks * MT + mt;
                        out[((size_t(pass) * NG + z / 4) * 64 + l) * 4 + z % 4] = T(v);
                    }
        }
        return 0;
    });
}

void tet3_mfma_fill_opsA(int P, const double *Dr, const double *Ds, const double *Dt, const double *LIFT,
                         float *out) {
    fill_opsA3<float>(P, Dr, Ds, Dt, LIFT, out);
}

void tet3_mfma_fill_opsA64(int P, const double *Dr, const double *Ds, const double *Dt, const double *LIFT,
                           double *out) {
    fill_opsA3<double>(P, Dr, Ds, Dt, LIFT, out);
}

template <typename T>
static hipError_t stage3_mfma(const Tet3Mesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                              bool bound, hipStream_t st) {
    Stage3MArgs<T> a;
    a.K = m.K;
    a.stage = stage;
    a.mode = rhs ? 0 : 1;
    a.g = T(m.gamma);
    a.ra = T(rk_a(stage));
    a.rb = T(rk_b(stage));
    a.Uin = static_cast<const T *>(Uin);
    a.Uout = static_cast<T *>(Uout);
    a.R = static_cast<T *>(R);
    a.rhs = static_cast<T *>(rhs);
    a.geo = static_cast<const T *>(m.fp32 ? static_cast<const void *>(m.geo32) : m.geo64);
    a.fmap = m.fmap;
    a.fmask = m.fmask;
    a.opsA = reinterpret_cast<const typename VT<T>::V4 *>(m.fp32 ? static_cast<const void *>(m.opsA)
                                                                  : static_cast<const void *>(m.opsA64));
    a.dt = m.scal + S_DT;
    a.bound = bound ? 1 : 0;
    a.gamma = m.gamma;
    a.vmax = m.vmax;
    a.flag = m.flag;
    return with_order3(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        using S = TetM<P>;
        const int blocks = (m.K + S::EB - 1) / S::EB;
        if constexpr (sizeof(T) == 4)
            hipLaunchKernelGGL((k_stage3_mfma<P>), dim3(blocks), dim3(S::NTH), 0, st, a);
        else
            hipLaunchKernelGGL((k_stage3_mfma64<P>), dim3(blocks), dim3(S::NTH), 0, st, a);
        return hipGetLastError();
    });
}

hipError_t launch_stage3(const Tet3Mesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                         bool bound, hipStream_t st) {
    return m.fp32 ? stage3_mfma<float>(m, Uin, Uout, R, rhs, stage, bound && !rhs, st)
                  : stage3_mfma<double>(m, Uin, Uout, R, rhs, stage, bound && !rhs, st);
}

hipError_t launch_bound3(const Tet3Mesh &m, const void *U, hipStream_t st) {
    return with_order3(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        const dim3 grid(tet3_blocks(m.K, P)), block(kB3);
        if (m.fp32)
            hipLaunchKernelGGL((k_cfl3<float, P>), grid, block, 0, st, m.K, m.gamma, static_cast<const float *>(U),
                               m.geo32, m.fmask, m.vmax, m.flag);
        else
            hipLaunchKernelGGL((k_cfl3<double, P>), grid, block, 0, st, m.K, m.gamma, static_cast<const double *>(U),
                               m.geo64, m.fmask, m.vmax, m.flag);
        return hipGetLastError();
    });
}

hipError_t launch_dt3(const Tet3Mesh &m, double dt_fixed, hipStream_t st) {
    hipLaunchKernelGGL(k_dt3, dim3(1), dim3(kSlots3), 0, st, m.cfl, dt_fixed, m.vmax, m.scal);
    return hipGetLastError();
}

}  // namespace dg
