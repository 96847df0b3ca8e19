// FP32 fused stage kernel on the matrix cores (gfx950, v_mfma_f32_16x16x4f32).
//
// For a straight (affine) element the metric terms are constants, so the
// volume term can be folded into the flux before the contraction:
//   -(r_x Dr F + s_x Ds F + r_y Dr G + s_y Ds G) = -Dr F' - Ds G',
//   F' = r_x F + r_y G,  G' = s_x F + s_y G,
// and the whole right-hand side of a field becomes one product
//   rhs = [-Dr  -Ds  LIFT] (Np x (2Np + 3Nfp))  .  [F'; G'; Fscale (n.F - F*)].
// The kernel forms that product for blocks of 4 elements x 4 fields = 16
// columns on the MFMA unit (A operand resident in VGPRs for the whole
// kernel, B operand staged in LDS).  A curved element keeps its per-node
// metrics: its F', G' rows are zeroed (the product then yields only the LIFT
// term) and its volume term is formed separately with per-node metrics on
// the vector ALUs.
//
// Memory: the element tile's state, the Runge-Kutta register and the
// outputs move as one coalesced 16-byte access per lane; per-element
// geometry (13 floats for an affine element) and connectivity (16 bytes)
// likewise; the only scattered reads are the neighbours' face traces.
// Blocks are remapped so that each XCD sweeps a contiguous range of tiles,
// which keeps recently loaded neighbours in that XCD's L2.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "launch.hpp"

namespace dg {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;

template <int P>
struct MShape {
    static constexpr int Np = (P + 1) * (P + 2) / 2;
    static constexpr int Nfp = P + 1;
    static constexpr int NF3 = 3 * Nfp;
    static constexpr int KV = 2 * Np + NF3;     // contraction length
    static constexpr int KS = (KV + 3) / 4;     // MFMA k-steps (K = 4 each)
    static constexpr int KP = 4 * KS;           // padded contraction length
    static constexpr int MT = (Np + 15) / 16;   // 16-row output tiles
    static constexpr int EW = 64 / Np;          // elements per wavefront (pointwise phase)
    static constexpr int EB = 4 * EW;           // elements per block
    static constexpr int NT = EB / 4;           // 16-column tiles per block
    static constexpr int TILE_FLOATS = EB * 4 * Np;   // state floats per block (<= 1024)
    static_assert(TILE_FLOATS <= 4 * kBlock, "one float4 per thread covers the tile");
};

struct MfmaArgs {
    int K, stage, mode, nblocks, chunk;
    float g, ra, rb;
    float qinf[4];
    const float *__restrict__ Uin;
    float *__restrict__ Uout;
    float *__restrict__ R;
    float *__restrict__ rhs;
    const int4 *__restrict__ conn;     // [K] {nbr0, nbr1, nbr2, packed face info}
    const float4 *__restrict__ geoA;   // [K][4]: rx sx ry sy | (nx ny Fscale) x 3 | pad
    const int *__restrict__ cidx;      // [K] curved slot or -1
    const float *__restrict__ geoC;    // [Kc][4 Np + 9 Nfp]
    const float *__restrict__ opsA;    // [MT][KS][64] A operand in lane order
    const float *__restrict__ ops;     // Dr | Ds (row-major) for curved elements
    const double *__restrict__ dt;
};

template <int P>
__global__ __launch_bounds__(kBlock) void k_stage_mfma(MfmaArgs a) {
    using S = MShape<P>;
    constexpr int Np = S::Np, Nfp = S::Nfp, NF3 = S::NF3, KS = S::KS, KP = S::KP, MT = S::MT;
    constexpr int EW = S::EW, EB = S::EB, NT = S::NT;
    // XCD-aware tile order: block b runs on XCD b % 8; give each XCD a
    // contiguous run of tiles.
    const int tile = (blockIdx.x % 8) * a.chunk + blockIdx.x / 8;
    if (tile >= a.nblocks) return;
    const long k0 = (long)tile * EB;
    const int nel = (int)min((long)EB, (long)a.K - k0);

    __shared__ float sU[EB * 4 * Np];
    __shared__ float sR[EB * 4 * Np];
    __shared__ float sB[NT][KP][16];
    __shared__ float sG[EB][16];
    __shared__ int sC[EB][4];
    __shared__ int sCurved[EB];
    __shared__ int sAny;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const long base = k0 * 4 * Np;
    const int nflt = nel * 4 * Np;

    // ---- coalesced tile loads: state, RK register, geometry, connectivity
    f32x4 u4 = {0, 0, 0, 0}, r4 = {0, 0, 0, 0};
    const bool flat_ok = 4 * tid < nflt;
    if (flat_ok) {
        u4 = *reinterpret_cast<const f32x4 *>(a.Uin + base + 4 * tid);
        if (a.mode && a.stage > 0) r4 = *reinterpret_cast<const f32x4 *>(a.R + base + 4 * tid);
    }
    if (tid < 4 * nel) {
        const float4 gv = a.geoA[k0 * 4 + tid];
        sG[tid >> 2][(tid & 3) * 4 + 0] = gv.x;
        sG[tid >> 2][(tid & 3) * 4 + 1] = gv.y;
        sG[tid >> 2][(tid & 3) * 4 + 2] = gv.z;
        sG[tid >> 2][(tid & 3) * 4 + 3] = gv.w;
    }
    if (tid < nel) {
        const int4 cv = a.conn[k0 + tid];
        sC[tid][0] = cv.x;
        sC[tid][1] = cv.y;
        sC[tid][2] = cv.z;
        sC[tid][3] = cv.w;
        sCurved[tid] = a.cidx[k0 + tid];
    }
    if (tid == 0) sAny = 0;
    if (flat_ok) *reinterpret_cast<f32x4 *>(&sU[4 * tid]) = u4;
    // zero the padded contraction rows of every column tile
    if constexpr (KP > S::KV) {
        constexpr int PADN = (KP - S::KV) * 16;
        for (int z = tid; z < NT * PADN; z += kBlock) {
            const int t = z / PADN, rem = z - t * PADN;
            sB[t][S::KV + rem / 16][rem % 16] = 0.f;
        }
    }
    // A operand for the whole kernel
    float A[MT][KS];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) A[mt][ks] = a.opsA[(mt * KS + ks) * 64 + lane];
    __syncthreads();

    // ---- pointwise fluxes (lane = element * Np + node within the wavefront)
    {
        const int le = lane / Np, i = lane - le * Np;
        const int el = wave * EW + le;
        if (le < EW && el < nel) {
            float u[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) u[c] = sU[(el * 4 + c) * Np + i];
            const float ir = 1.f / u[0];
            const float vx = u[1] * ir, vy = u[2] * ir;
            const float p = pressure(a.g, u);
            const float F[4] = {u[1], u[1] * vx + p, u[2] * vx, (u[3] + p) * vx};
            const float G[4] = {u[2], u[1] * vy, u[2] * vy + p, (u[3] + p) * vy};
            const int t = el >> 2, col = (el & 3) * 4;
            f32x4 f, gg;
            if (sCurved[el] < 0) {
                const float rx = sG[el][0], sx = sG[el][1], ry = sG[el][2], sy = sG[el][3];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    f[c] = rx * F[c] + ry * G[c];
                    gg[c] = sx * F[c] + sy * G[c];
                }
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    f[c] = F[c];
                    gg[c] = G[c];
                }
                sAny = 1;
            }
            *reinterpret_cast<f32x4 *>(&sB[t][i][col]) = f;
            *reinterpret_cast<f32x4 *>(&sB[t][Np + i][col]) = gg;
        }
    }
    // ---- face gather and Lax-Friedrichs flux (task = element * 3Nfp + face node)
    for (int task = tid; task < nel * NF3; task += kBlock) {
        const int el = task / NF3, q = task - el * NF3;
        const int f = q / Nfp, j = q - f * Nfp;
        const int vm = face_node(P, f, j);
        float um[4], up[4], d[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) um[c] = sU[(el * 4 + c) * Np + vm];
        float nx, ny, fs;
        const int cs = sCurved[el];
        if (cs < 0) {
            nx = sG[el][4 + 3 * f];
            ny = sG[el][5 + 3 * f];
            fs = sG[el][6 + 3 * f];
        } else {
            const float *gc = a.geoC + (long)cs * (4 * Np + 9 * Nfp) + 4 * Np;
            nx = gc[q];
            ny = gc[NF3 + q];
            fs = gc[2 * NF3 + q];
        }
        const int info = sC[el][3];
        const int code = face_bc(info, f);
        if (code == BC_INTERIOR) {
            const long kn = sC[el][f];
            const int vp = face_node(P, face_nbr_face(info, f), Nfp - 1 - j);
            const long ln = kn - k0;
            if (ln >= 0 && ln < nel) {
#pragma unroll
                for (int c = 0; c < 4; ++c) up[c] = sU[(ln * 4 + c) * Np + vp];
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) up[c] = a.Uin[(kn * 4 + c) * Np + vp];
            }
        } else {
            ghost_state(a.g, code, um, nx, ny, a.qinf, up);
        }
        lf_jump(a.g, um, up, nx, ny, d);
        f32x4 jv = {fs * d[0], fs * d[1], fs * d[2], fs * d[3]};
        *reinterpret_cast<f32x4 *>(&sB[el >> 2][2 * Np + q][(el & 3) * 4]) = jv;
    }
    __syncthreads();

    // ---- curved elements: volume term with per-node metrics (VALU), then
    // clear their F/G rows so the product contributes only the LIFT term
    if (sAny) {
        const int le = lane / Np, i = lane - le * Np;
        const int el = wave * EW + le;
        const bool curved = le < EW && el < nel && sCurved[el] >= 0;
        if (curved) {
            const float *gc = a.geoC + (long)sCurved[el] * (4 * Np + 9 * Nfp);
            const float rx = gc[i], sx = gc[Np + i], ry = gc[2 * Np + i], sy = gc[3 * Np + i];
            const int t = el >> 2, col = (el & 3) * 4;
            float drf[4] = {0, 0, 0, 0}, dsf[4] = {0, 0, 0, 0}, drg[4] = {0, 0, 0, 0},
                  dsg[4] = {0, 0, 0, 0};
            for (int j = 0; j < Np; ++j) {
                const float dr = a.ops[i * Np + j], ds = a.ops[Np * Np + i * Np + j];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float fv = sB[t][j][col + c], gv = sB[t][Np + j][col + c];
                    drf[c] += dr * fv;
                    dsf[c] += ds * fv;
                    drg[c] += dr * gv;
                    dsg[c] += ds * gv;
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c)
                sR[(el * 4 + c) * Np + i] = -(rx * drf[c] + sx * dsf[c] + ry * drg[c] + sy * dsg[c]);
        }
        __syncthreads();
        if (curved) {
            const int t = el >> 2, col = (el & 3) * 4;
            const f32x4 z = {0, 0, 0, 0};
            *reinterpret_cast<f32x4 *>(&sB[t][i][col]) = z;
            *reinterpret_cast<f32x4 *>(&sB[t][Np + i][col]) = z;
        }
        __syncthreads();
    }

    // ---- the contraction on the matrix cores: wave w takes column tiles
    // w, w+4, ...; result row m = node, column n = 4 * element + field
    for (int t = wave; t < NT; t += 4) {
        f32x4 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const float b = sB[t][4 * ks + (lane >> 4)][lane & 15];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[mt][ks], b, acc[mt], 0, 0, 0);
        }
        const int el = t * 4 + ((lane & 15) >> 2), c = lane & 3;
        if (el < nel) {
            const bool add = sCurved[el] >= 0;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 16 * mt + 4 * (lane >> 4) + r;
                    if (i < Np) {
                        float *dst = &sR[(el * 4 + c) * Np + i];
                        *dst = add ? *dst + acc[mt][r] : acc[mt][r];
                    }
                }
        }
    }
    __syncthreads();

    // ---- epilogue: Runge-Kutta update (or the bare rhs), coalesced
    if (flat_ok) {
        const f32x4 rh = *reinterpret_cast<const f32x4 *>(&sR[4 * tid]);
        if (a.mode == 0) {
            *reinterpret_cast<f32x4 *>(a.rhs + base + 4 * tid) = rh;
        } else {
            const float dt = float(*a.dt);
            f32x4 rn;
            if (a.stage == 0)
                rn = dt * rh;
            else
                rn = a.ra * r4 + dt * rh;
            *reinterpret_cast<f32x4 *>(a.R + base + 4 * tid) = rn;
            *reinterpret_cast<f32x4 *>(a.Uout + base + 4 * tid) = u4 + a.rb * rn;
        }
    }
}

template <int P>
void fill_opsA(const double *Dr, const double *Ds, const double *LIFT, float *out) {
    using S = MShape<P>;
    constexpr int Np = S::Np, NF3 = S::NF3;
    for (int mt = 0; mt < S::MT; ++mt)
        for (int ks = 0; ks < S::KS; ++ks)
            for (int l = 0; l < 64; ++l) {
                const int m = 16 * mt + (l & 15), k = 4 * ks + (l >> 4);
                double v = 0.0;
                if (m < Np) {
                    if (k < Np)
                        v = -Dr[m * Np + k];
                    else if (k < 2 * Np)
                        v = -Ds[m * Np + (k - Np)];
                    else if (k < S::KV)
                        v = LIFT[m * NF3 + (k - 2 * Np)];
                }
                out[(mt * S::KS + ks) * 64 + l] = float(v);
            }
}

template <typename F>
auto with_order_m(int P, F &&f) {
    switch (P) {
        case 1: return f(std::integral_constant<int, 1>());
        case 2: return f(std::integral_constant<int, 2>());
        case 3: return f(std::integral_constant<int, 3>());
        case 4: return f(std::integral_constant<int, 4>());
        default: return f(std::integral_constant<int, 5>());
    }
}

}  // namespace

size_t mfma_opsA_floats(int P) {
    return with_order_m(P, [](auto PC) {
        using S = MShape<decltype(PC)::value>;
        return size_t(S::MT) * S::KS * 64;
    });
}

void mfma_fill_opsA(int P, const double *Dr, const double *Ds, const double *LIFT, float *out) {
    with_order_m(P, [&](auto PC) {
        fill_opsA<decltype(PC)::value>(Dr, Ds, LIFT, out);
        return 0;
    });
}

int mfma_elements_per_block(int P) {
    return with_order_m(P, [](auto PC) { return MShape<decltype(PC)::value>::EB; });
}

hipError_t launch_stage_mfma(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs,
                             int stage, hipStream_t st) {
    MfmaArgs a;
    a.K = m.K;
    a.stage = stage;
    a.mode = rhs ? 0 : 1;
    a.g = float(m.gamma);
    a.ra = float(rk_a(stage));
    a.rb = float(rk_b(stage));
    for (int c = 0; c < 4; ++c) a.qinf[c] = float(m.qinf[c]);
    a.Uin = static_cast<const float *>(Uin);
    a.Uout = static_cast<float *>(Uout);
    a.R = static_cast<float *>(R);
    a.rhs = static_cast<float *>(rhs);
    a.conn = reinterpret_cast<const int4 *>(m.conn4);
    a.geoA = reinterpret_cast<const float4 *>(m.geoA);
    a.cidx = m.cidx;
    a.geoC = m.geoC;
    a.opsA = m.opsA;
    a.ops = m.ops32;
    a.dt = m.scal + S_DT;
    return with_order_m(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        using S = MShape<P>;
        a.nblocks = (m.K + S::EB - 1) / S::EB;
        a.chunk = (a.nblocks + 7) / 8;
        hipLaunchKernelGGL((k_stage_mfma<P>), dim3(8 * a.chunk), dim3(kBlock), 0, st, a);
        return hipGetLastError();
    });
}

}  // namespace dg
