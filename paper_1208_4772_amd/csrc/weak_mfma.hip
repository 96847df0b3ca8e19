// The over-integrated weak form (Section 2, eqs. stiffness, mass, face_mass,
// semidiscrete) on the matrix cores, for FP32 handles whose elements are all
// straight.  There M_k = J M_ref, so
//
//   dU/dt = (1/J) M_ref^-1 [Drc^T a + Dsc^T b - L s],
//   a_q = w_q J (r_x F + r_y G)(x_q),  b_q = w_q J (s_x F + s_y G)(x_q),
//   s_g = w_g sJ F*(u-, u+)(x_g),
//
// with Drc, Dsc the derivatives of the nodal basis at the cubature points and
// L the transpose of the interpolation from face nodes to face Gauss points
// (each face's block scattered onto that face's nodes).  A block takes 16
// elements; each wavefront owns a group of four (16 columns, element-major,
// the four fields of an element adjacent) and runs two products for it:
//   1. the state at the cubature points, Icub (NQ x Np) . U (Np x 16);
//   2. the update, A2 (Np x (2 NQ + 3 NG)) . [a; b; s] (x 16), with
//      A2 = M_ref^-1 [Drc^T | Dsc^T | -L] formed in FP64 on the host.
// Fluxes at the cubature and Gauss points run on the VALUs between the two,
// one thread per point.  The operators are A fragments of
// v_mfma_f32_16x16x4f32 (lane l holds row 16 mt + (l & 15), column
// 4 ks + (l >> 4); zero outside the matrix), read from the caches.
#include <hip/hip_runtime.h>

#include <vector>

#include "common.hpp"
#include "launch.hpp"

namespace dg {
namespace {

typedef float wf32x4 __attribute__((ext_vector_type(4)));

constexpr int kWMBlock = 256;

template <int P>
struct WMShape {
    static constexpr int Np = (P + 1) * (P + 2) / 2, Nfp = P + 1;
    static constexpr int n = (3 * P + 2) / 2, NQ = n * n, NG = n, NFG = 3 * NG;
    static constexpr int KS1 = (Np + 3) / 4, MT1 = (NQ + 15) / 16;
    static constexpr int K2 = 2 * NQ + NFG, KS2 = (K2 + 3) / 4, MT2 = (Np + 15) / 16;
    // LDS column strides (words) of the two B operands, 4 (mod 8) so that
    // the 16 columns a row of lanes reads fall in different banks
    static constexpr int S1 = (4 * KS1) % 8 == 4 ? 4 * KS1 : 4 * KS1 + 4;
    static constexpr int S2 = (4 * KS2) % 8 == 4 ? 4 * KS2 : 4 * KS2 + 4;
    static constexpr int NFRAG = MT1 * KS1 + MT2 * KS2;
    static constexpr int EB = 16;   // elements per block: four per wavefront
    static_assert(16 * MT1 <= S2, "the cubature values fit a column of the second operand");
    static_assert(EB * 4 * Np <= EB * 4 * S2, "the result fits the second operand's buffer");
};

struct WeakMArgs {
    int K, stage, mode, riemann;
    float g, ra, rb;
    FarField<float> ff;
    const float *__restrict__ Uin;
    float *__restrict__ Uout;
    float *__restrict__ R;
    float *__restrict__ rhs;
    const int *__restrict__ nbr;
    const int *__restrict__ finfo;
    const float *__restrict__ opsA;   // [NFRAG][64]: product 1's fragments (mt, ks), then product 2's
    const float *__restrict__ wq;     // [NQ] cubature weights
    const float *__restrict__ If;     // [NG][Nfp] face nodes -> Gauss points
    const float *__restrict__ geoA;   // [K][5] r_x s_x r_y s_y J
    const float *__restrict__ geoF;   // [K][3][NG][3] n_x n_y w_g sJ
    const double *__restrict__ dt;
};

template <int P>
__global__ __launch_bounds__(kWMBlock) void k_stage_weak_mfma(WeakMArgs a) {
    using S = WMShape<P>;
    constexpr int Np = S::Np, Nfp = S::Nfp, NQ = S::NQ, NG = S::NG, NFG = S::NFG, EB = S::EB;
    constexpr int S1 = S::S1, S2 = S::S2, KS1 = S::KS1, MT1 = S::MT1, KS2 = S::KS2, MT2 = S::MT2, K2 = S::K2;
    __shared__ __attribute__((aligned(16))) float sU[EB * 4][S1];
    __shared__ __attribute__((aligned(16))) float sB[EB * 4][S2];
    const long k0 = (long)blockIdx.x * EB;
    const int nel = (int)min((long)EB, (long)a.K - k0);
    const int tid = threadIdx.x, lane = tid & 63, c0 = (tid >> 6) * 16;
    const int col = lane & 15, kq = lane >> 4;

    // the state tile, column (element, field) by column; zero in the
    // padding rows and for elements beyond the mesh
    for (int z = tid; z < EB * 4 * S1; z += kWMBlock) {
        const int cz = z / S1, j = z - cz * S1;
        float v = 0.f;
        if (j < Np && (cz >> 2) < nel) v = a.Uin[(k0 * 4 + cz) * Np + j];
        (&sU[0][0])[z] = v;
    }
    __syncthreads();

    // product 1: the state at the cubature points, into sB[column][q]
    {
        wf32x4 acc[MT1];
#pragma unroll
        for (int mt = 0; mt < MT1; ++mt) acc[mt] = wf32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS1; ++ks) {
            const float b = sU[c0 + col][4 * ks + kq];
#pragma unroll
            for (int mt = 0; mt < MT1; ++mt)
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.opsA[(mt * KS1 + ks) * 64 + lane], b, acc[mt], 0,
                                                               0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < MT1; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) sB[c0 + col][16 * mt + 4 * kq + r] = acc[mt][r];
    }
    __syncthreads();

    // fluxes: the weighted contravariant volume fluxes at the cubature
    // points and w_g sJ (n.F(u-) - F*) at the face Gauss points, held in
    // registers until every thread has read the cubature values
    constexpr int NV = (EB * NQ + kWMBlock - 1) / kWMBlock;
    constexpr int NF = (EB * NFG + kWMBlock - 1) / kWMBlock;
    float va[NV][kFields], vb[NV][kFields], vs[NF][kFields];
#pragma unroll
    for (int t = 0; t < NV; ++t) {
        const int z = tid + kWMBlock * t;
        const int el = z / NQ, q = z - el * NQ;
#pragma unroll
        for (int c = 0; c < kFields; ++c) va[t][c] = vb[t][c] = 0.f;
        if (z < EB * NQ && el < nel) {
            float u[kFields];
#pragma unroll
            for (int c = 0; c < kFields; ++c) u[c] = sB[el * 4 + c][q];
            const float ir = rcp(u[0]);
            const float vx = u[1] * ir, vy = u[2] * ir, p = pressure_ir(a.g, u, ir);
            const float F[kFields] = {u[1], u[1] * vx + p, u[2] * vx, (u[3] + p) * vx};
            const float G[kFields] = {u[2], u[1] * vy, u[2] * vy + p, (u[3] + p) * vy};
            const float *gk = a.geoA + (k0 + el) * 5;
            const float wJ = a.wq[q] * gk[4];
            const float wrx = wJ * gk[0], wsx = wJ * gk[1], wry = wJ * gk[2], wsy = wJ * gk[3];
#pragma unroll
            for (int c = 0; c < kFields; ++c) {
                va[t][c] = wrx * F[c] + wry * G[c];
                vb[t][c] = wsx * F[c] + wsy * G[c];
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        const int z = tid + kWMBlock * t;
        const int el = z / NFG, fg = z - el * NFG, f = fg / NG, gq = fg - f * NG;
#pragma unroll
        for (int c = 0; c < kFields; ++c) vs[t][c] = 0.f;
        if (z < EB * NFG && el < nel) {
            const long k = k0 + el;
            float um[kFields] = {}, up[kFields] = {};
            for (int j = 0; j < Nfp; ++j) {
                const float l = a.If[gq * Nfp + j];
                const int v = face_node(P, f, j);
#pragma unroll
                for (int c = 0; c < kFields; ++c) um[c] += l * sU[el * 4 + c][v];
            }
            const float *gf = a.geoF + ((k * 3 + f) * NG + gq) * 3;
            const float nx = gf[0], ny = gf[1], ws = gf[2];
            const int info = a.finfo[k];
            const int code = face_bc(info, f);
            if (code == BC_INTERIOR) {
                // the neighbour's face node Nfp-1-j sits on this face's node j
                const long kn = a.nbr[k * 3 + f];
                const int fn = face_nbr_face(info, f);
                for (int j = 0; j < Nfp; ++j) {
                    const float l = a.If[gq * Nfp + j];
                    const int v = face_node(P, fn, Nfp - 1 - j);
#pragma unroll
                    for (int c = 0; c < kFields; ++c) up[c] += l * a.Uin[(kn * kFields + c) * Np + v];
                }
            } else {
                ghost_state(a.g, code, um, nx, ny, a.ff, up);
            }
            float fm[kFields], lm, d[kFields];
            normal_flux(a.g, um, nx, ny, fm, lm);
            flux_jump(a.riemann, a.g, um, up, nx, ny, d);
#pragma unroll
            for (int c = 0; c < kFields; ++c) vs[t][c] = ws * (fm[c] - d[c]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NV; ++t) {
        const int z = tid + kWMBlock * t;
        if (z < EB * NQ) {
            const int el = z / NQ, q = z - el * NQ;
#pragma unroll
            for (int c = 0; c < kFields; ++c) {
                sB[el * 4 + c][q] = va[t][c];
                sB[el * 4 + c][NQ + q] = vb[t][c];
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        const int z = tid + kWMBlock * t;
        if (z < EB * NFG) {
            const int el = z / NFG, fg = z - el * NFG;
#pragma unroll
            for (int c = 0; c < kFields; ++c) sB[el * 4 + c][2 * NQ + fg] = vs[t][c];
        }
    }
    constexpr int PAD = 4 * KS2 - K2;
    if constexpr (PAD > 0) {
        for (int z = tid; z < EB * 4 * PAD; z += kWMBlock) sB[z / PAD][K2 + z % PAD] = 0.f;
    }
    __syncthreads();

    // product 2: M_ref^-1 (V - S) for the wavefront's 16 columns
    wf32x4 acc2[MT2];
#pragma unroll
    for (int mt = 0; mt < MT2; ++mt) acc2[mt] = wf32x4{0.f, 0.f, 0.f, 0.f};
    const float *A2 = a.opsA + MT1 * KS1 * 64;
#pragma unroll
    for (int ks = 0; ks < KS2; ++ks) {
        const float b = sB[c0 + col][4 * ks + kq];
#pragma unroll
        for (int mt = 0; mt < MT2; ++mt)
            acc2[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(A2[(mt * KS2 + ks) * 64 + lane], b, acc2[mt], 0, 0, 0);
    }
    // every wavefront has read its columns: the buffer now takes the
    // result in the state's own order ([element][field][node])
    __syncthreads();
    {
        const int el = (c0 + col) >> 2;
        const float J = el < nel ? a.geoA[(k0 + el) * 5 + 4] : 1.f;
        float *o = &sB[0][0];
#pragma unroll
        for (int mt = 0; mt < MT2; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * mt + 4 * kq + r;
                if (i < Np) o[(c0 + col) * Np + i] = acc2[mt][r] / J;
            }
    }
    __syncthreads();
    const float *o = &sB[0][0];
    const float dt = a.mode ? float(*a.dt) : 0.f;
    for (int z = tid; z < nel * 4 * Np; z += kWMBlock) {
        const long idx = k0 * 4 * Np + z;
        const float val = o[z];
        if (a.mode == 0) {
            a.rhs[idx] = val;
        } else {
            const int cz = z / Np, i = z - cz * Np;
            const float rr = (a.stage == 0) ? dt * val : a.ra * a.R[idx] + dt * val;
            a.R[idx] = rr;
            a.Uout[idx] = sU[cz][i] + a.rb * rr;
        }
    }
}

template <typename F>
hipError_t with_order_wm(int P, F &&f) {
    switch (P) {
        case 1: return f(std::integral_constant<int, 1>());
        case 2: return f(std::integral_constant<int, 2>());
        case 3: return f(std::integral_constant<int, 3>());
        case 4: return f(std::integral_constant<int, 4>());
        case 5: return f(std::integral_constant<int, 5>());
        default: return hipErrorInvalidValue;
    }
}

template <int P>
void fill_weak_opsA(const double *Icub, const double *Drc, const double *Dsc, const double *If,
                    const double *Minv, float *out) {
    using S = WMShape<P>;
    constexpr int Np = S::Np, Nfp = S::Nfp, NQ = S::NQ, NG = S::NG, NFG = S::NFG, K2 = S::K2;
    // L [Np][3 NG]: face f's Gauss point g takes If[g][j] from face node j
    std::vector<double> L(size_t(Np) * NFG, 0.0);
    for (int f = 0; f < 3; ++f)
        for (int j = 0; j < Nfp; ++j)
            for (int g = 0; g < NG; ++g) L[size_t(face_node(P, f, j)) * NFG + f * NG + g] = If[g * Nfp + j];
    // A2 = M_ref^-1 [Drc^T | Dsc^T | -L], FP64
    std::vector<double> A2(size_t(Np) * K2, 0.0);
    for (int i = 0; i < Np; ++i)
        for (int kk = 0; kk < K2; ++kk) {
            double s = 0.0;
            for (int m = 0; m < Np; ++m) {
                const double v = kk < NQ ? Drc[kk * Np + m]
                                         : (kk < 2 * NQ ? Dsc[(kk - NQ) * Np + m] : -L[size_t(m) * NFG + kk - 2 * NQ]);
                s += Minv[i * Np + m] * v;
            }
            A2[size_t(i) * K2 + kk] = s;
        }
    auto frag = [&](int rows, int cols, auto &&at, int MT, int KS, float *dst) {
        for (int mt = 0; mt < MT; ++mt)
            for (int ks = 0; ks < KS; ++ks)
                for (int l = 0; l < 64; ++l) {
                    const int row = 16 * mt + (l & 15), kk = 4 * ks + (l >> 4);
                    dst[(size_t(mt) * KS + ks) * 64 + l] = (row < rows && kk < cols) ? float(at(row, kk)) : 0.f;
                }
    };
    frag(NQ, Np, [&](int r, int c) { return Icub[r * Np + c]; }, S::MT1, S::KS1, out);
    frag(Np, K2, [&](int r, int c) { return A2[size_t(r) * K2 + c]; }, S::MT2, S::KS2, out + S::MT1 * S::KS1 * 64);
}

}  // namespace

size_t weak_mfma_opsA_values(int P) {
    size_t n = 0;
    with_order_wm(P, [&](auto PC) {
        n = size_t(WMShape<decltype(PC)::value>::NFRAG) * 64;
        return hipSuccess;
    });
    return n;
}

void weak_mfma_fill_opsA(int P, const double *Icub, const double *Drc, const double *Dsc, const double *If,
                         const double *Minv, float *out) {
    with_order_wm(P, [&](auto PC) {
        fill_weak_opsA<decltype(PC)::value>(Icub, Drc, Dsc, If, Minv, out);
        return hipSuccess;
    });
}

hipError_t launch_stage_weak_mfma(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                                  hipStream_t st) {
    if (!m.fp32 || !m.wopsA || m.wKc != 0) return hipErrorInvalidValue;
    return with_order_wm(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        using S = WMShape<P>;
        WeakMArgs a;
        a.K = m.K;
        a.stage = stage;
        a.mode = rhs ? 0 : 1;
        a.riemann = m.riemann;
        a.g = float(m.gamma);
        a.ra = float(rk_a(stage));
        a.rb = float(rk_b(stage));
        a.ff = make_farfield<float>(m.gamma, m.qinf);
        a.Uin = static_cast<const float *>(Uin);
        a.Uout = static_cast<float *>(Uout);
        a.R = static_cast<float *>(R);
        a.rhs = static_cast<float *>(rhs);
        a.nbr = m.nbr;
        a.finfo = m.finfo;
        a.opsA = m.wopsA;
        // the FP32 operator table: Icub | Drc | Dsc | wq | If | Minv
        a.wq = m.wops32 + size_t(3) * S::NQ * S::Np;
        a.If = a.wq + S::NQ;
        a.geoA = m.wgeoA32;
        a.geoF = m.wgeoF32;
        a.dt = m.scal + S_DT;
        const dim3 grid(unsigned((m.K + S::EB - 1) / S::EB)), block(kWMBlock);
        hipLaunchKernelGGL((k_stage_weak_mfma<P>), grid, block, 0, st, a);
        return hipGetLastError();
    });
}

}  // namespace dg
