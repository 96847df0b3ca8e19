// FP32 fused stage kernel on the matrix cores (gfx950, v_mfma_f32_16x16x4f32).
//
// For a straight (affine) element the metric terms are constants, so the
// volume term can be folded into the flux before the contraction:
//   -(r_x Dr F + s_x Ds F + r_y Dr G + s_y Ds G) = -Dr F' - Ds G',
//   F' = r_x F + r_y G,  G' = s_x F + s_y G,
// and the whole right-hand side of a field becomes one product
//   rhs = [-Dr  -Ds  LIFT] (Np x (2Np + 3Nfp))  .  [F'; G'; Fscale (n.F - F*)].
// The kernel forms that product for groups of 4 elements x 4 fields = 16
// columns on the MFMA unit (A operand read from global memory, where the
// same few KB serve every block from the caches; B operand built in LDS).
// A curved element keeps its per-node metrics: its F', G' rows are zeroed
// (the product then yields only the LIFT term) and its volume term is
// formed separately with per-node metrics on the VALUs.
//
// Memory: the element tile's state, the Runge-Kutta register and the
// outputs move as one coalesced 16-byte access per lane; per-element
// geometry (13 floats for an affine element) and connectivity (16 bytes)
// likewise; the only scattered reads are the neighbours' face traces, which
// each thread issues at the start for the face nodes it will handle, so that
// their latency overlaps the tile load and the pointwise phase.  Blocks are
// remapped so that each XCD sweeps a contiguous range of tiles, which keeps
// recently loaded neighbours in that XCD's L2.  LDS per block is kept small
// (the result is staged in the B operand's own space) so that several
// blocks share a CU and hide each other's memory latency.
//
// Time step: in a fused run without viscosity the last stage also reduces
// the CFL bound of the new state (FP64 per node from the FP32 state, exact
// maximum) into device slots, and the next step's first stage turns it into dt (FP64), so
// a step needs no separate reduction launches; with viscosity the first
// stage's sensor fills the slots instead (it knows the new viscosity).
#include <hip/hip_runtime.h>

#include <cstring>

#include "common.hpp"
#include "launch.hpp"

namespace dg {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;   // default waves per workgroup (the autotuner may pick 2 or 8)
constexpr int default_waves(int) { return kWaves; }
constexpr int kCurvedBit = 1 << 12;   // in the packed face-info word

// BF3: the product runs as three BF16 products (v_mfma_f32_16x16x32_bf16)
// of hi/lo splits, K padded to multiples of 32.  W: wavefronts per
// workgroup (the elements per workgroup are W times those of a wavefront).
template <int P, bool BF3 = false, int W = kWaves>
struct MShape {
    static constexpr int Np = (P + 1) * (P + 2) / 2;
    static constexpr int Nfp = P + 1;
    static constexpr int NF3 = 3 * Nfp;
    static constexpr int KV = 2 * Np + NF3;     // contraction length
    static constexpr int KS = (KV + 3) / 4;     // FP32 MFMA k-steps (K = 4 each)
    static constexpr int KS32 = (KV + 31) / 32; // BF16 MFMA k-steps (K = 32 each)
    static constexpr int KP = BF3 ? 32 * KS32 : 4 * KS;  // padded contraction length
    static constexpr int MT = (Np + 15) / 16;   // 16-row output tiles
    static constexpr int EW = 64 / Np;          // elements per wavefront (pointwise phase)
    static constexpr int NTH = 64 * W;          // threads per block
    static constexpr int EB = W * EW;           // elements per block
    static constexpr int NT = (EB + 3) / 4;     // 16-column groups per block
    static constexpr int TF = EB * 4 * Np;      // state floats per block
    static constexpr int TPT = (EB * NF3 + NTH - 1) / NTH;  // face-node tasks per thread
    static constexpr int GPT = (4 * EB + NTH - 1) / NTH;    // geometry float4 per thread
    static_assert(TF <= 4 * NTH, "one float4 per thread covers the tile");
    static_assert(EB <= NTH, "one thread per element loads the connectivity");
    static_assert(16 * Np <= 16 * KP, "a column group's result fits in its B block");
};

struct MfmaArgs {
    int K, stage, mode, nblocks, chunk;
    int riemann;     // numerical flux: RIEMANN_LF or RIEMANN_HLLC
    int cfl_mode;    // 1: this (first) stage turns *vmax_in into dt
    int cfl_accum;   // 1: this (last) stage reduces the new state's CFL bound into *vmax_out
    float g, ra, rb;
    FarField<float> ff;
    double gamma, cfl, dt_fixed;
    const float *__restrict__ Uin;
    float *__restrict__ Uout;
    float *__restrict__ R;
    float *__restrict__ rhs;
    const int4 *__restrict__ conn;     // [K] {nbr0, nbr1, nbr2, packed face info}
    const float4 *__restrict__ geoA;   // [K][4]: rx sx ry sy | (nx ny Fscale) x 3 | pad
    const int *__restrict__ cidx;      // [K] curved slot or -1
    const int *__restrict__ cpre;      // [K + 1] curved elements before element k
    const float *__restrict__ geoC;    // [Kc][4 Np + 9 Nfp]
    const float *__restrict__ opsA;    // [MT][KS][64] A operand in lane order
    const float *__restrict__ ops;     // Dr | Ds (row-major) for curved elements
    const float *__restrict__ eps;     // [K] artificial viscosity (viscous handles)
    const float *__restrict__ Q;       // [K][2][4][Np] sqrt(eps) grad U (viscous handles)
    double *__restrict__ scal;
    const unsigned long long *__restrict__ vmax_in;
    unsigned long long *__restrict__ vmax_out;
    int *__restrict__ flag;
};

// Node id of face node j of face f without branches (selects only).
template <int P>
__device__ __forceinline__ int face_node_sel(int f, int j) {
    const int n = f == 0 ? 0 : (f == 1 ? j : P - j);
    const int off = f == 0 ? j : (f == 1 ? P - j : 0);
    return n * (P + 1) - ((n * (n - 1)) >> 1) + off;
}

// Lax-Friedrichs face term of one face-node task, scaled by Fscale, into the
// B operand.  CURVED: the tile holds curved elements, whose normals and
// Fscale are per face node.
template <int P, bool BF3, int W, bool CURVED, bool AV>
__device__ __forceinline__ void face_task(const MfmaArgs &a, const long k0, const int el, const int q,
                                          const float (&upn)[4], const float *sU, const float (*sG)[16],
                                          const int4 cv, const int *sFN, float *sBflat) {
    using S = MShape<P, BF3, W>;
    constexpr int Np = S::Np, Nfp = S::Nfp, NF3 = S::NF3, KP = S::KP;
    const int f = q / Nfp;
    const int vm = sFN[q];
    float um[4], up[4], d[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) um[c] = sU[(el * 4 + c) * Np + vm];
    float nx, ny, fs;
    if (CURVED && (cv.w & kCurvedBit)) {
        const float *gc = a.geoC + (long)a.cidx[k0 + el] * (4 * Np + 9 * Nfp) + 4 * Np;
        nx = gc[q];
        ny = gc[NF3 + q];
        fs = gc[2 * NF3 + q];
    } else {
        nx = sG[el][4 + 3 * f];
        ny = sG[el][5 + 3 * f];
        fs = sG[el][6 + 3 * f];
    }
    const int code = face_bc(cv.w, f);
    if (code == BC_INTERIOR) {
#pragma unroll
        for (int c = 0; c < 4; ++c) up[c] = upn[c];
    } else {
        ghost_state(a.g, code, um, nx, ny, a.ff, up);
    }
    if (a.riemann == RIEMANN_HLLC) {
        hllc_jump(a.g, um, up, nx, ny, d);
    } else {
        // local Lax-Friedrichs: n.F(U-) - F* = (n.F(U-) - n.F(U+)) / 2 + lam (U+ - U-) / 2
        float fm[4], fp[4], lm, lp;
        normal_flux(a.g, um, nx, ny, fm, lm);
        normal_flux(a.g, up, nx, ny, fp, lp);
        const float lam = lm > lp ? lm : lp;
#pragma unroll
        for (int c = 0; c < 4; ++c) d[c] = 0.5f * (fm[c] - fp[c]) + 0.5f * lam * (up[c] - um[c]);
    }
    if constexpr (AV) {
        // viscous face term (sigma Q)* . n - (sigma Q)- . n: (sigma Q)* the
        // mean of both sides inside, the mirror closure at a slip wall
        // (wall_visc_jump), the interior value at the far field (so no
        // contribution there)
        if (code == BC_INTERIOR) {
            const int j = q - f * Nfp;
            const long km = k0 + el;
            const long kn = f == 0 ? cv.x : (f == 1 ? cv.y : cv.z);
            const int vp = sFN[face_nbr_face(cv.w, f) * Nfp + Nfp - 1 - j];
            const float sm = fsqrt(a.eps[km]), sp = fsqrt(a.eps[kn]);
            const float *Qm = a.Q + km * 8 * Np, *Qp = a.Q + kn * 8 * Np;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float vmv = sm * (nx * Qm[c * Np + vm] + ny * Qm[(4 + c) * Np + vm]);
                const float vpv = sp * (nx * Qp[c * Np + vp] + ny * Qp[(4 + c) * Np + vp]);
                d[c] += 0.5f * (vmv + vpv) - vmv;
            }
        } else if (code == BC_WALL) {
            const long km = k0 + el;
            const float sm = fsqrt(a.eps[km]);
            const float *Qm = a.Q + km * 8 * Np;
            float vmv[4], vj[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) vmv[c] = sm * (nx * Qm[c * Np + vm] + ny * Qm[(4 + c) * Np + vm]);
            wall_visc_jump(vmv, nx, ny, vj);
#pragma unroll
            for (int c = 0; c < 4; ++c) d[c] += vj[c];
        }
    }
    const f32x4 jv = {fs * d[0], fs * d[1], fs * d[2], fs * d[3]};
    *reinterpret_cast<f32x4 *>(&sBflat[((el >> 2) * KP + 2 * Np + q) * 16 + (el & 3) * 4]) = jv;
}

// Time-step bound and state check of node `in` of an element of an FP32
// matrix-core handle: the state widened to FP64, its wave speed times the
// largest Fscale of the faces the node lies on (the element's FP32 record:
// g16[6 + 3 f] for an affine element, the per-face-node values of its curved
// record gc otherwise), all in FP64 (cfl_bound).
template <int P>
__device__ __forceinline__ double node_cfl(double gamma, const float (&uf)[4], int in, const float *g16,
                                           const float *gc, int &bad) {
    constexpr int Np = (P + 1) * (P + 2) / 2, Nfp = P + 1, NF3 = 3 * Nfp;
    double u[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] = double(uf[c]);
    constexpr NodeFaceTable<P> kNF;
    const int nq = kNF.v[in];
    // an interior node (on no face) takes Fscale 0: only its state check
    float fs = 0.f;
    if (nq) {
        const int q0 = (nq & 255) - 1, q1 = (nq >> 8) - 1;
        if (!gc) {
            fs = g16[6 + 3 * (q0 / Nfp)];
            if (q1 >= 0) fs = fmaxf(fs, g16[6 + 3 * (q1 / Nfp)]);
        } else {
            const float *gf = gc + 4 * Np + 2 * NF3;
            fs = gf[q0];
            if (q1 >= 0) fs = fmaxf(fs, gf[q1]);
        }
    }
    return cfl_bound_checked(gamma, u, double(fs), 0.0, P + 1.0, bad);
}

// One tile (EB consecutive elements) of one mesh.  `a` may live in kernel
// arguments (single mesh) or in a device job table (batched meshes); its
// fields are uniform across the block.
template <int P, bool BF3, int W, bool AV>
__device__ __forceinline__ void stage_tile(const MfmaArgs &a, const int tile) {
    using S = MShape<P, BF3, W>;
    constexpr int NTH = S::NTH;
    constexpr int Np = S::Np, Nfp = S::Nfp, NF3 = S::NF3, KS = S::KS, KS32 = S::KS32, KP = S::KP, MT = S::MT;
    constexpr int EW = S::EW, EB = S::EB, NT = S::NT, TF = S::TF, TPT = S::TPT, GPT = S::GPT;

    // ---- time step of this stage, requested now: the first stage of a step
    // reduces the CFL-bound slots (after the first barrier, when they have
    // arrived), the others read the step the first one booked
    unsigned long long vb = 0;
    double dtd = 0.0;
    if (a.cfl_mode)
        vb = a.vmax_in[threadIdx.x & (kVmaxSlots - 1)];
    else if (a.mode)
        dtd = a.scal[S_DT];

    const long k0 = (long)tile * EB;
    const int nel = (int)min((long)EB, (long)a.K - k0);
    // whether the tile holds a curved element (uniform: two scalar loads)
    const bool any_curved = a.cpre[k0 + nel] != a.cpre[k0];

    __shared__ float sU[TF];
    __shared__ float sB[NT][KP][16];    // B operand; afterwards the result of that column group
    __shared__ float sG[EB][16];
    __shared__ double sRed[W];
    __shared__ int sFN[NF3];              // face node ids, face-major, counter-clockwise

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const long base = k0 * 4 * Np;
    const int nflt = nel * 4 * Np;
    const int ntask = nel * NF3;
    // result (element el, field c, node i) lives in its column group's block
    auto res = [&](int el, int off) -> float & { return (&sB[el >> 2][0][0])[(el & 3) * 4 * Np + off]; };

    // ---- loads.  Every address is clamped into the tile so that the loads
    // need no branches.  Order matters: a wavefront's memory counter retires
    // loads in issue order, so what the first barrier needs (the tile and
    // its geometry) goes first, then the neighbour face traces for the
    // face-node tasks this thread will handle (task = element * 3 Nfp + face
    // node; tasks tid, tid + 64 W, ...; needed in the face phase), then the
    // Runge-Kutta register (needed in the epilogue): the last two stay in
    // flight across the barrier and the pointwise phase.
    int4 tconn[TPT];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int task = min(tid + t * NTH, ntask - 1);
        tconn[t] = a.conn[k0 + task / NF3];
    }
    const bool flat_ok = 4 * tid < nflt;
    const f32x4 u4 = *reinterpret_cast<const f32x4 *>(a.Uin + base + (flat_ok ? 4 * tid : 0));
    // geometry records, four float4 per element: where a tile holds more
    // elements than a quarter of the threads (P = 1), a thread loads two
    float4 g4[GPT];
#pragma unroll
    for (int t = 0; t < GPT; ++t) g4[t] = a.geoA[k0 * 4 + min(tid + t * NTH, 4 * nel - 1)];
    float upn[TPT][4];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int task = min(tid + t * NTH, ntask - 1);
        const int q = task % NF3, f = q / Nfp, j = q - f * Nfp;
        const int4 cv = tconn[t];
        const bool inner = face_bc(cv.w, f) == BC_INTERIOR;
        const int kn = inner ? (f == 0 ? cv.x : (f == 1 ? cv.y : cv.z)) : int(k0);
        const int vp = face_node_sel<P>(face_nbr_face(cv.w, f), Nfp - 1 - j);
        const float *src = a.Uin + (long)kn * 4 * Np + vp;
#pragma unroll
        for (int c = 0; c < 4; ++c) upn[t][c] = src[c * Np];
    }
    f32x4 r4 = {0, 0, 0, 0};
    if (a.mode && a.stage > 0) r4 = *reinterpret_cast<const f32x4 *>(a.R + base + (flat_ok ? 4 * tid : 0));

    if (tid < NF3) sFN[tid] = face_node_sel<P>(tid / Nfp, tid % Nfp);
    if constexpr (KP > S::KV) {
        constexpr int PADN = (KP - S::KV) * 16;
        for (int z = tid; z < NT * PADN; z += NTH) {
            const int t = z / PADN, rem = z - t * PADN;
            sB[t][S::KV + rem / 16][rem % 16] = 0.f;
        }
    }
#pragma unroll
    for (int t = 0; t < GPT; ++t)
        if (tid + t * NTH < 4 * nel) reinterpret_cast<float4 *>(&sG[0][0])[tid + t * NTH] = g4[t];
    if (flat_ok) *reinterpret_cast<f32x4 *>(&sU[4 * tid]) = u4;
    __syncthreads();

    if (a.cfl_mode) {
        // the bound is the maximum over the slots (non-negative doubles order
        // like their bit patterns); every wavefront reduces them itself
        for (int off = kVmaxSlots / 2; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(vb, off);
            vb = o > vb ? o : vb;
        }
        const double vmax = __longlong_as_double((long long)vb);
        dtd = a.dt_fixed > 0.0 ? a.dt_fixed : a.cfl * (1.0 / vmax);
        if (tile == 0 && threadIdx.x < kVmaxSlots) {
            if (threadIdx.x == 0) {
                a.scal[S_DT] = dtd;
                a.scal[S_T] += dtd;
                a.scal[S_DTMIN] = dtd < a.scal[S_DTMIN] ? dtd : a.scal[S_DTMIN];
                a.scal[S_DTMAX] = dtd > a.scal[S_DTMAX] ? dtd : a.scal[S_DTMAX];
                a.scal[S_STEPS] += 1.0;
            }
            a.vmax_out[threadIdx.x] = 0ull;
        }
        // the same in every lane: keep it in scalar registers
        const unsigned long long db = (unsigned long long)__double_as_longlong(dtd);
        const unsigned lo = __builtin_amdgcn_readfirstlane(unsigned(db));
        const unsigned hi = __builtin_amdgcn_readfirstlane(unsigned(db >> 32));
        dtd = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    }

    // ---- pointwise fluxes (lane = element * Np + node within the wavefront)
    const int le = lane / Np, in = lane - le * Np;
    const int eln = wave * EW + le;
    const bool node_ok = le < EW && eln < nel;
    bool curved_lane = false;
    if (node_ok) {
        float u[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) u[c] = sU[(eln * 4 + c) * Np + in];
        const float ir = rcp(u[0]);
        const float vx = u[1] * ir, vy = u[2] * ir;
        const float p = pressure_ir(a.g, u, ir);
        float F[4] = {u[1], u[1] * vx + p, u[2] * vx, (u[3] + p) * vx};
        float G[4] = {u[2], u[1] * vy, u[2] * vy + p, (u[3] + p) * vy};
        if constexpr (AV) {
            // viscous flux sigma Q (sigma = sqrt(eps) per element)
            const float sig = fsqrt(a.eps[k0 + eln]);
            const float *Qe = a.Q + (k0 + eln) * 8 * Np;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                F[c] -= sig * Qe[c * Np + in];
                G[c] -= sig * Qe[(4 + c) * Np + in];
            }
        }
        const int t = eln >> 2, col = (eln & 3) * 4;
        f32x4 f, gg;
        curved_lane = any_curved && sG[eln][13] != 0.f;
        if (!curved_lane) {
            const float rx = sG[eln][0], sx = sG[eln][1], ry = sG[eln][2], sy = sG[eln][3];
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
        }
        *reinterpret_cast<f32x4 *>(&sB[t][in][col]) = f;
        *reinterpret_cast<f32x4 *>(&sB[t][Np + in][col]) = gg;
    }
    // no barrier: the face phase reads only the tile's state, geometry and
    // connectivity, and writes other rows of the B operand than the fluxes

    // ---- Lax-Friedrichs flux at the face nodes
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int task = tid + t * NTH;
        if (task < ntask) {
            const int el = task / NF3, q = task - el * NF3;
            if (any_curved)
                face_task<P, BF3, W, true, AV>(a, k0, el, q, upn[t], sU, sG, tconn[t], sFN, &sB[0][0][0]);
            else
                face_task<P, BF3, W, false, AV>(a, k0, el, q, upn[t], sU, sG, tconn[t], sFN, &sB[0][0][0]);
        }
    }
    // the A operand of the product (the same few KB for every block, so it
    // comes from the caches; FP32: four fragments per lane per 16-byte load;
    // BF16x3: hi and lo splits).  A tile without curved elements requests it
    // before the barrier, so that its latency overlaps the other
    // wavefronts' face tasks; a curved tile after its volume phase, which
    // needs the registers.  At P = 5 the operand (30 fragments per lane)
    // does not fit the register budget that early, and is requested just
    // before the product.
    constexpr bool early_A = P <= 4;
    constexpr int NZ = MT * KS, NG4 = (NZ + 3) / 4;
    f32x4 ga4[BF3 ? 1 : NG4];
    u32x4 ah[BF3 ? MT * KS32 : 1], al[BF3 ? MT * KS32 : 1];
    auto load_A = [&]() {
        if (wave < NT) {
            if constexpr (!BF3) {
                const f32x4 *ga = reinterpret_cast<const f32x4 *>(a.opsA);
#pragma unroll
                for (int g = 0; g < NG4; ++g) ga4[g] = ga[g * 64 + lane];
            } else {
                const u32x4 *opsB = reinterpret_cast<const u32x4 *>(a.opsA);
#pragma unroll
                for (int z = 0; z < MT * KS32; ++z) {
                    ah[z] = opsB[(2 * z) * 64 + lane];
                    al[z] = opsB[(2 * z + 1) * 64 + lane];
                }
            }
        }
    };
    if (early_A && !any_curved) load_A();
    __syncthreads();

    // ---- curved elements: volume term with per-node metrics (VALU), kept
    // in registers; their F/G rows are then cleared so the product gives
    // only the LIFT term
    float vol[4] = {0, 0, 0, 0};
    if (any_curved) {
        if (curved_lane) {
            const float *gc = a.geoC + (long)a.cidx[k0 + eln] * (4 * Np + 9 * Nfp);
            const float rx = gc[in], sx = gc[Np + in], ry = gc[2 * Np + in], sy = gc[3 * Np + in];
            const int t = eln >> 2, col = (eln & 3) * 4;
            float drf[4] = {0, 0, 0, 0}, dsf[4] = {0, 0, 0, 0}, drg[4] = {0, 0, 0, 0},
                  dsg[4] = {0, 0, 0, 0};
#pragma unroll 1
            for (int j = 0; j < Np; ++j) {
                const float dr = a.ops[in * Np + j], ds = a.ops[Np * Np + in * Np + j];
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
            for (int c = 0; c < 4; ++c) vol[c] = -(rx * drf[c] + sx * dsf[c] + ry * drg[c] + sy * dsg[c]);
        }
        __syncthreads();
        if (curved_lane) {
            const int t = eln >> 2, col = (eln & 3) * 4;
            const f32x4 z = {0, 0, 0, 0};
            *reinterpret_cast<f32x4 *>(&sB[t][in][col]) = z;
            *reinterpret_cast<f32x4 *>(&sB[t][Np + in][col]) = z;
        }
        if (early_A) load_A();
        __syncthreads();
    }
    if (!early_A) load_A();

    // ---- the contraction on the matrix cores: wave w takes column groups
    // w, w+4, ...; result row = node, column = 4 * element + field.  The
    // wavefront writes the result over its own (fully consumed) B block.
    for (int t = wave; t < NT; t += W) {
        f32x4 acc[MT], acc2[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            acc[mt] = f32x4{0, 0, 0, 0};
            acc2[mt] = f32x4{0, 0, 0, 0};
        }
        if constexpr (!BF3) {
            // two independent accumulation chains per output tile (even and
            // odd k-steps) halve the dependent-MFMA latency
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const float b = sB[t][4 * ks + (lane >> 4)][lane & 15];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    if (ks & 1)
                        acc2[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga4[(mt * KS + ks) / 4][(mt * KS + ks) % 4], b,
                                                                        acc2[mt], 0, 0, 0);
                    else
                        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga4[(mt * KS + ks) / 4][(mt * KS + ks) % 4], b,
                                                                       acc[mt], 0, 0, 0);
                }
            }
        } else {
            // BF16x3: A = Ah + Al (split on the host), B = Bh + Bl (split
            // here, round to nearest even), AB ~ Ah Bh + (Ah Bl + Al Bh); the
            // dropped Al Bl and the split residues are O(2^-16) |A||B|.
            // Lane l holds k-slots 8 (l / 16) + i, i < 8, of row/column l % 16
            // in both operands, so the slot-to-k assignment is the same on
            // both sides of the product.
#pragma unroll
            for (int ks = 0; ks < KS32; ++ks) {
                bf16x8 bh, bl;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float b = sB[t][32 * ks + 8 * (lane >> 4) + i][lane & 15];
                    bh[i] = __bf16(b);
                    bl[i] = __bf16(b - float(bh[i]));
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const bf16x8 Ah = __builtin_bit_cast(bf16x8, ah[mt * KS32 + ks]);
                    const bf16x8 Al = __builtin_bit_cast(bf16x8, al[mt * KS32 + ks]);
                    acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, bh, acc[mt], 0, 0, 0);
                    acc2[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, bl, acc2[mt], 0, 0, 0);
                    acc2[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, bh, acc2[mt], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] += acc2[mt];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int el = t * 4 + ((lane & 15) >> 2), c = lane & 3;
        if (el < nel) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 16 * mt + 4 * (lane >> 4) + r;
                    if (i < Np) res(el, c * Np + i) = acc[mt][r];
                }
        }
    }
    __syncthreads();
    if (any_curved) {
        if (curved_lane) {
#pragma unroll
            for (int c = 0; c < 4; ++c) res(eln, c * Np + in) += vol[c];
        }
        __syncthreads();
    }

    // ---- epilogue: Runge-Kutta update (or the bare rhs), coalesced
    const int fe = (4 * tid) / (4 * Np), foff = 4 * tid - fe * 4 * Np;
    if (flat_ok) {
        const f32x4 rh = *reinterpret_cast<const f32x4 *>(&res(fe, foff));
        if (a.mode == 0) {
            *reinterpret_cast<f32x4 *>(a.rhs + base + 4 * tid) = rh;
        } else {
            const float dt = float(dtd);
            const f32x4 rn = a.stage == 0 ? dt * rh : a.ra * r4 + dt * rh;
            // the stage's input state, still in LDS (kept there rather than in
            // registers through the product)
            const f32x4 un = *reinterpret_cast<const f32x4 *>(&sU[4 * tid]) + a.rb * rn;
            *reinterpret_cast<f32x4 *>(a.R + base + 4 * tid) = rn;
            *reinterpret_cast<f32x4 *>(a.Uout + base + 4 * tid) = un;
            if (a.cfl_accum) *reinterpret_cast<f32x4 *>(&sU[4 * tid]) = un;
        }
    }
    if (a.cfl_accum) {
        // CFL bound and state check of the new state: one lane per node
        // (node_cfl), reduced into the block's slot; the next step's first
        // stage turns the maximum into dt
        __syncthreads();
        double vmax_lane = 0.0;
        int bad = 0;
        if (node_ok) {
            float u[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) u[c] = sU[(eln * 4 + c) * Np + in];
            const float *gc = curved_lane ? a.geoC + (long)a.cidx[k0 + eln] * (4 * Np + 9 * Nfp) : nullptr;
            vmax_lane = node_cfl<P>(a.gamma, u, in, &sG[eln][0], gc, bad);
        }
        if (__any(bad) && lane == 0) atomicOr(a.flag, 1);
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(vmax_lane, off);
            vmax_lane = o > vmax_lane ? o : vmax_lane;
        }
        if (lane == 0) sRed[wave] = vmax_lane;
        __syncthreads();
        if (tid == 0) {
            double m = sRed[0];
            for (int w = 1; w < W; ++w) m = sRed[w] > m ? sRed[w] : m;
            // non-negative doubles order like their bit patterns
            atomicMax(a.vmax_out + (blockIdx.x & (kVmaxSlots - 1)), (unsigned long long)__double_as_longlong(m));
        }
    }
}

// First-step CFL bound of a matrix-core handle: the same node_cfl over every
// node of the state, reduced into the slots (which the caller has zeroed),
// so that a run's first step takes the bound a fused last stage would have
// left (dg_run(N) twice equals dg_run(2N)).
template <int P>
__global__ __launch_bounds__(256) void k_cfl_vmax_mfma(int K, double gamma, const float *__restrict__ U,
                                                       const int4 *__restrict__ conn,
                                                       const float4 *__restrict__ geoA,
                                                       const int *__restrict__ cidx,
                                                       const float *__restrict__ geoC,
                                                       unsigned long long *__restrict__ slots,
                                                       int *__restrict__ flag) {
    constexpr int Np = (P + 1) * (P + 2) / 2, Nfp = P + 1;
    __shared__ double sRed[4];
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    const long k = idx / Np;
    const int in = int(idx - k * Np);
    double v = 0.0;
    int bad = 0;
    if (k < K) {
        float u[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) u[c] = U[(k * 4 + c) * Np + in];
        float g16[16];
#pragma unroll
        for (int z = 0; z < 4; ++z) {
            const float4 r = geoA[k * 4 + z];
            g16[4 * z] = r.x;
            g16[4 * z + 1] = r.y;
            g16[4 * z + 2] = r.z;
            g16[4 * z + 3] = r.w;
        }
        const bool curved = (conn[k].w & kCurvedBit) != 0;
        const float *gc = curved ? geoC + (long)cidx[k] * (4 * Np + 9 * Nfp) : nullptr;
        v = node_cfl<P>(gamma, u, in, g16, gc, bad);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sRed[0];
        for (int w = 1; w < 4; ++w) m = sRed[w] > m ? sRed[w] : m;
        atomicMax(slots + (blockIdx.x & (kVmaxSlots - 1)), (unsigned long long)__double_as_longlong(m));
    }
}

// XCD-aware block order: block b runs on XCD b % 8; each XCD gets a
// contiguous run of work items.
__device__ __forceinline__ int xcd_item(int chunk) { return (blockIdx.x % 8) * chunk + blockIdx.x / 8; }

// Occupancy request: as many resident waves per SIMD as the LDS allows (at
// most 8), which caps the registers per lane at 512 / waves; the kernel
// hides its memory latency with resident waves.
template <int P, bool BF3, int W, bool AV = false>
constexpr int waves_per_simd() {
    using S = MShape<P, BF3, W>;
    constexpr int lds = S::TF * 4 + S::NT * S::KP * 64 + S::EB * 64 + 256;
    constexpr int blocks = (160 * 1024) / lds;      // resident blocks per CU by LDS
    constexpr int waves = blocks * W / 4;           // per SIMD
    // the BF16x3 product holds its hi/lo operand fragments in registers, and
    // the viscous terms need more too: at most 6 waves (85 registers) there,
    // so that nothing spills
    constexpr int cap = (BF3 || AV) ? 6 : 8;
    return waves >= cap ? cap : (waves < 1 ? 1 : waves);
}

template <int P, bool BF3, int W, bool AV>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(waves_per_simd<P, BF3, W, AV>())))
void k_stage_mfma(MfmaArgs a) {
    const int tile = xcd_item(a.chunk);
    if (tile >= a.nblocks) return;
    stage_tile<P, BF3, W, AV>(a, tile);
}

// Batched meshes of one order: work item = (job, tile); a job is one mesh's
// argument record for this stage.
template <int P, bool BF3, int W, bool AV>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(waves_per_simd<P, BF3, W, AV>())))
void k_stage_mfma_batch(const MfmaArgs *__restrict__ jobs, const int2 *__restrict__ items,
                        const int *__restrict__ nitems_dev) {
    // one work item per workgroup; the grid covers the list's capacity and
    // the length is read from device memory, so a captured launch stays
    // valid while the list changes.  XCD x (block b runs on XCD b % 8) takes
    // the x-th contiguous eighth of the items present; surplus blocks exit.
    // (A loop over several items per workgroup raised the register count
    // enough to spill: every value derived from the thread index was hoisted
    // out of it.)
    const int n = *nitems_dev;
    const int per = (n + 7) / 8, i = int(blockIdx.x / 8);
    const int w = int(blockIdx.x % 8) * per + i;
    if (i >= per || w >= n) return;
    const int2 it = items[w];
    stage_tile<P, BF3, W, AV>(jobs[it.x], it.y);
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
                // lane l's fragments z = mt KS + ks, four per 16-byte group
                const int z = mt * S::KS + ks;
                out[((z / 4) * 64 + l) * 4 + z % 4] = float(v);
            }
}

// Round to nearest even into BF16 (finite inputs).
inline unsigned short bf16_rne(float f) {
    unsigned u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
inline double bf16_value(unsigned short h) {
    const unsigned u = unsigned(h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// BF16x3 A operand: per (output tile, 32-wide k-step) a hi block and a lo
// block of 64 lanes x 8 BF16 values; lane l, slot i holds row 16 mt + l % 16,
// column 32 ks + 8 (l / 16) + i; two slots per 32-bit word, low half first.
template <int P>
void fill_opsB(const double *Dr, const double *Ds, const double *LIFT, unsigned *out) {
    using S = MShape<P, true>;
    constexpr int Np = S::Np, NF3 = S::NF3;
    for (int mt = 0; mt < S::MT; ++mt)
        for (int ks = 0; ks < S::KS32; ++ks)
            for (int l = 0; l < 64; ++l)
                for (int w = 0; w < 4; ++w) {
                    unsigned short hv[2], lv[2];
                    for (int h = 0; h < 2; ++h) {
                        const int m = 16 * mt + (l & 15), k = 32 * ks + 8 * (l >> 4) + 2 * w + h;
                        double v = 0.0;
                        if (m < Np) {
                            if (k < Np)
                                v = -Dr[m * Np + k];
                            else if (k < 2 * Np)
                                v = -Ds[m * Np + (k - Np)];
                            else if (k < S::KV)
                                v = LIFT[m * NF3 + (k - 2 * Np)];
                        }
                        hv[h] = bf16_rne(float(v));
                        lv[h] = bf16_rne(float(v - bf16_value(hv[h])));
                    }
                    const int z = mt * S::KS32 + ks;
                    out[((2 * z) * 64 + l) * 4 + w] = unsigned(hv[0]) | unsigned(hv[1]) << 16;
                    out[((2 * z + 1) * 64 + l) * 4 + w] = unsigned(lv[0]) | unsigned(lv[1]) << 16;
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
        return size_t((S::MT * S::KS + 3) / 4) * 4 * 64;
    });
}

void mfma_fill_opsA(int P, const double *Dr, const double *Ds, const double *LIFT, float *out) {
    with_order_m(P, [&](auto PC) {
        fill_opsA<decltype(PC)::value>(Dr, Ds, LIFT, out);
        return 0;
    });
}

size_t mfma_opsB_words(int P) {
    return with_order_m(P, [](auto PC) {
        using S = MShape<decltype(PC)::value, true>;
        return size_t(S::MT) * S::KS32 * 2 * 64 * 4;
    });
}

void mfma_fill_opsB(int P, const double *Dr, const double *Ds, const double *LIFT, unsigned *out) {
    with_order_m(P, [&](auto PC) {
        fill_opsB<decltype(PC)::value>(Dr, Ds, LIFT, out);
        return 0;
    });
}

// Dispatch on the waves per workgroup (2, 4 or 8; 0 = the default).
template <typename F>
auto with_waves(int w, F &&f) {
    switch (w) {
        case 2: return f(std::integral_constant<int, 2>());
        case 8: return f(std::integral_constant<int, 8>());
        default: return f(std::integral_constant<int, kWaves>());
    }
}

int mfma_elements_per_block(int P, int waves) {
    return with_order_m(P, [&](auto PC) {
        return with_waves(waves, [&](auto WC) {
            return MShape<decltype(PC)::value, false, decltype(WC)::value>::EB;
        });
    });
}

int mfma_curved_bit() { return kCurvedBit; }

int mfma_default_waves() { return kWaves; }

static MfmaArgs make_args(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                          const MfmaStep &step, int waves, const void *eps = nullptr,
                          const void *Q = nullptr) {
    MfmaArgs a;
    a.K = m.K;
    a.riemann = m.riemann;
    a.stage = stage;
    a.mode = rhs ? 0 : 1;
    a.cfl_mode = step.cfl_mode;
    a.cfl_accum = step.cfl_accum;
    a.g = float(m.gamma);
    a.ra = float(rk_a(stage));
    a.rb = float(rk_b(stage));
    a.ff = make_farfield<float>(m.gamma, m.qinf);
    a.gamma = m.gamma;
    a.cfl = m.cfl;
    a.dt_fixed = step.dt_fixed;
    a.Uin = static_cast<const float *>(Uin);
    a.Uout = static_cast<float *>(Uout);
    a.R = static_cast<float *>(R);
    a.rhs = static_cast<float *>(rhs);
    a.conn = reinterpret_cast<const int4 *>(m.conn4);
    a.geoA = reinterpret_cast<const float4 *>(m.geoA);
    a.cidx = m.cidx;
    a.cpre = m.cpre;
    a.geoC = m.geoC;
    a.opsA = m.bf3 ? reinterpret_cast<const float *>(m.opsB) : m.opsA;
    a.ops = m.ops32;
    a.eps = static_cast<const float *>(eps);
    a.Q = static_cast<const float *>(Q);
    a.scal = m.scal;
    a.vmax_in = step.vmax_in;
    a.vmax_out = step.vmax_out;
    a.flag = m.flag;
    const int eb = mfma_elements_per_block(m.P, waves);
    a.nblocks = (m.K + eb - 1) / eb;
    a.chunk = (a.nblocks + 7) / 8;
    return a;
}

size_t mfma_args_bytes() { return sizeof(MfmaArgs); }

// A batch group runs one workgroup shape (waves per workgroup) for all its
// meshes: records and tiles are made with the group's shape.
void mfma_fill_args(const DevMesh &m, const void *Uin, void *Uout, void *R, int stage, const MfmaStep &step,
                    int waves, void *out, const void *eps, const void *Q) {
    const MfmaArgs a = make_args(m, Uin, Uout, R, nullptr, stage, step, waves, eps, Q);
    std::memcpy(out, &a, sizeof(a));
}

int mfma_tiles(const DevMesh &m, int waves) {
    const int eb = mfma_elements_per_block(m.P, waves);
    return (m.K + eb - 1) / eb;
}

hipError_t launch_stage_mfma_batch(int P, bool bf3, bool av, int waves, const void *jobs, const void *items,
                                   const int *nitems_dev, int capacity, hipStream_t st) {
    if (capacity <= 0) return hipSuccess;
    const auto *j = static_cast<const MfmaArgs *>(jobs);
    const auto *it = static_cast<const int2 *>(items);
    return with_order_m(P, [&](auto PC) {
        constexpr int PP = decltype(PC)::value;
        return with_waves(waves, [&](auto WC) {
            constexpr int W = decltype(WC)::value;
            const dim3 grid(unsigned((capacity + 7) / 8 * 8)), block(64 * W);
            if (bf3 && av)
                hipLaunchKernelGGL((k_stage_mfma_batch<PP, true, W, true>), grid, block, 0, st, j, it, nitems_dev);
            else if (bf3)
                hipLaunchKernelGGL((k_stage_mfma_batch<PP, true, W, false>), grid, block, 0, st, j, it,
                                   nitems_dev);
            else if (av)
                hipLaunchKernelGGL((k_stage_mfma_batch<PP, false, W, true>), grid, block, 0, st, j, it,
                                   nitems_dev);
            else
                hipLaunchKernelGGL((k_stage_mfma_batch<PP, false, W, false>), grid, block, 0, st, j, it,
                                   nitems_dev);
            return hipGetLastError();
        });
    });
}

hipError_t launch_cfl_vmax_mfma(const DevMesh &m, const void *U, unsigned long long *slots, hipStream_t st) {
    hipError_t e = hipMemsetAsync(slots, 0, kVmaxSlots * sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    return with_order_m(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        constexpr int Np = (P + 1) * (P + 2) / 2;
        const long nodes = long(m.K) * Np;
        const dim3 grid(unsigned((nodes + 255) / 256)), block(256);
        hipLaunchKernelGGL((k_cfl_vmax_mfma<P>), grid, block, 0, st, m.K, m.gamma,
                           static_cast<const float *>(U), reinterpret_cast<const int4 *>(m.conn4),
                           reinterpret_cast<const float4 *>(m.geoA), m.cidx, m.geoC, slots, m.flag);
        return hipGetLastError();
    });
}

hipError_t launch_stage_mfma(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs,
                             int stage, const MfmaStep &step, hipStream_t st, const void *eps, const void *Q) {
    const int waves = m.waves_per_block ? m.waves_per_block : default_waves(m.P);
    if (m.av && (!eps || !Q)) return hipErrorInvalidValue;
    MfmaArgs a = make_args(m, Uin, Uout, R, rhs, stage, step, waves, eps, Q);
    return with_order_m(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        return with_waves(waves, [&](auto WC) {
            constexpr int W = decltype(WC)::value;
            const dim3 grid(8 * a.chunk), block(64 * W);
            if (m.av) {
                if (m.bf3)
                    hipLaunchKernelGGL((k_stage_mfma<P, true, W, true>), grid, block, 0, st, a);
                else
                    hipLaunchKernelGGL((k_stage_mfma<P, false, W, true>), grid, block, 0, st, a);
            } else {
                if (m.bf3)
                    hipLaunchKernelGGL((k_stage_mfma<P, true, W, false>), grid, block, 0, st, a);
                else
                    hipLaunchKernelGGL((k_stage_mfma<P, false, W, false>), grid, block, 0, st, a);
            }
            return hipGetLastError();
        });
    });
}

}  // namespace dg
