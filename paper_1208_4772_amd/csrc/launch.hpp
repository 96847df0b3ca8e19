// Interface between the C-ABI layer and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

namespace dg {

// The fused CFL bound is reduced into this many slots per parity (workgroup
// b uses slot b % kVmaxSlots), so that its atomics do not all hit one
// address; the next step's first stage takes the maximum of the slots.
constexpr int kVmaxSlots = 64;

// Slots of the per-mesh FP64 device scalars.
enum Scalar {
    S_DT = 0,       // step of the current/last step
    S_T = 1,        // simulated time accumulated since the last reset
    S_DTMIN = 2,
    S_DTMAX = 3,
    S_TOT = 4,      // 4 totals
    S_RES = 8,      // 4 residuals
    S_STEPS = 12,
    S_NSCAL = 16
};

struct DevMesh {
    int K = 0, P = 0, Np = 0, Nfp = 0;
    bool fp32 = false;
    bool bf3 = false;              // FP32 handle whose stage product runs as BF16x3
    bool av = false;
    int riemann = 0;               // numerical flux: 0 local Lax-Friedrichs, 1 HLLC
    bool weak = false;             // the over-integrated weak form instead of the nodal form
    // weak-form tables (weak.hip): operators Icub | Drc | Dsc | wq | If | Minv,
    // straight-element metrics [K][5], face data [K][3][NG][3], curved
    // elements' mapped cubature weights [Kc][NQ][4] and inverse mass matrices
    const double *wops64 = nullptr, *wgeoA64 = nullptr, *wgeoF64 = nullptr, *wgeoC64 = nullptr,
                 *wminv64 = nullptr;
    const float *wops32 = nullptr, *wgeoA32 = nullptr, *wgeoF32 = nullptr, *wgeoC32 = nullptr,
                *wminv32 = nullptr;
    const int *widx = nullptr;     // [K] curved slot of the weak-form tables or -1
    const float *wopsA = nullptr;  // FP32 handles of straight elements: the weak form's matrix-core
                                   // operator fragments (weak_mfma.hip)
    int wKc = 0;
    double gamma = 1.4, cfl = 0.5;
    double qinf[4] = {1, 0, 0, 2.5};
    double av_s0 = 0, av_kappa = 1;
    const int *nbr = nullptr;      // [K][3] neighbour element
    const int *finfo = nullptr;    // [K] packed neighbour face and bc codes
    // FP64 tables
    const double *geo64 = nullptr;   // [K][4][Np] rx, sx, ry, sy
    const double *fgeo64 = nullptr;  // [K][3][3*Nfp] nx, ny, Fscale
    const double *wmass = nullptr;   // [K][Np] mass weights w_ki = sum_j M_ij J_kj
    const double *emax64 = nullptr;  // [K] eps_max per element
    const double *ops64 = nullptr;   // Dr | Ds | LIFT | Vinv
    // FP32 tables (FP32 handles)
    const float *geo32 = nullptr, *fgeo32 = nullptr, *emax32 = nullptr, *ops32 = nullptr;
    // FP32 matrix-core stage kernel tables
    const int *conn4 = nullptr;     // [K][4] nbr0, nbr1, nbr2, packed face info
    const float *geoA = nullptr;    // [K][16] affine geometry record
    const int *cidx = nullptr;      // [K] curved slot or -1
    const int *cpre = nullptr;      // [K + 1] number of curved elements before element k
    const float *geoC = nullptr;    // [Kc][4 Np + 9 Nfp] curved geometry
    const float *opsA = nullptr;    // MFMA A operand table
    const double *opsA64 = nullptr; // FP64 handles of straight elements without viscosity: the
                                    // FP64 matrix-core stage's A operand (null: the VALU stage)
    const double *geoA64 = nullptr; // ... and its [K][16] geometry records (k_pack_affine64)
    const unsigned *opsB = nullptr; // BF16x3 A operand table (hi and lo splits)
    int Kc = 0;
    int ncu = 256;                  // compute units of the device
    int waves_per_block = 0;        // stage-kernel workgroup shape: 2, 4 or 8 wavefronts (0: the order's default)
    unsigned long long *vmax = nullptr;   // [2][kVmaxSlots] CFL-bound slots (FP64 bit patterns)
    // device scalars and reduction scratch
    double *scal = nullptr;   // [S_NSCAL]
    int *flag = nullptr;      // non-finite / non-positive state flag
    int *count = nullptr;     // setup counters (bad J, bad normals)
    double *partial = nullptr;
    int npartial = 0;
};

// FP64 stage on the matrix cores (stage64.hip): A operand [LIFT -Dr -Ds] in
// lane order, and the launch
size_t mfma64_opsA_values(int P);
void mfma64_fill_opsA(int P, const double *Dr, const double *Ds, const double *LIFT, double *out);
// bound: a run's step-closing stage, which also reduces the next step's
// time-step bound into m.vmax (first kVmaxSlots slots) and checks the state
hipError_t launch_stage_mfma64(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                               bool bound, hipStream_t st);
// dt from the bound in m.vmax's slots (or the fixed step); clears them
hipError_t launch_dt_slots64(const DevMesh &m, double dt_fixed, hipStream_t st);
hipError_t launch_pack_affine64(const DevMesh &m, double *rec, hipStream_t st);

// offsets of the operators in the ops tables
inline size_t ops_size(int Np, int Nfp) { return size_t(Np) * Np * 3 + size_t(Np) * 3 * Nfp; }
inline size_t off_Dr(int, int) { return 0; }
inline size_t off_Ds(int Np, int) { return size_t(Np) * Np; }
inline size_t off_LIFT(int Np, int) { return size_t(2) * Np * Np; }
inline size_t off_Vinv(int Np, int Nfp) { return size_t(2) * Np * Np + size_t(Np) * 3 * Nfp; }

// number of partial-reduction slots the reduction kernels need
int partial_slots(int K, int P);

// setup: FP64 geometric factors from node coordinates (device x, y
// [K][Np]); counts J <= 0 nodes into count[0].
hipError_t launch_geometry(const DevMesh &m, const double *x, const double *y, double *geo64,
                           double *fgeo64, double *wmass, double *emax64, double av_eps0,
                           hipStream_t st);
// counts interior face nodes whose normal is not minus the neighbour's into count[1]
hipError_t launch_check_normals(const DevMesh &m, hipStream_t st);
hipError_t launch_cast(const double *src, float *dst, size_t n, hipStream_t st);

// rhs of state U (mode 0) or one LSERK stage (mode 1):
//   R = a_s R + dt rhs (stage 0: R = dt rhs), Uout = Uin + b_s R.
// eps: [K] viscosities and Q: [K][2][4][Np] gradients (AV only).
hipError_t launch_stage(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs,
                        int stage, const void *eps, const void *Q, hipStream_t st);
// Time-step handling of one matrix-core stage launch.
struct MfmaStep {
    int cfl_mode = 0;      // 1: first stage computes dt from *vmax_in (and books it)
    int cfl_accum = 0;     // 1: last stage reduces the new state's CFL bound into *vmax_out
    double dt_fixed = 0.0; // > 0 overrides the CFL step when cfl_mode = 1
    const unsigned long long *vmax_in = nullptr;
    unsigned long long *vmax_out = nullptr;
};
// FP32 matrix-core stage kernel (no artificial viscosity)
hipError_t launch_stage_mfma(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                             const MfmaStep &step, hipStream_t st, const void *eps = nullptr,
                             const void *Q = nullptr);
int mfma_curved_bit();
// batched meshes: per-(mesh, stage) argument records in device memory and a
// work list of (record, tile) items, all meshes of order P
size_t mfma_args_bytes();
void mfma_fill_args(const DevMesh &m, const void *Uin, void *Uout, void *R, int stage, const MfmaStep &step,
                    int waves, void *out, const void *eps = nullptr, const void *Q = nullptr);
int mfma_tiles(const DevMesh &m, int waves);
int mfma_default_waves();
// Batched launches: one work item per workgroup over a list whose length
// the kernels read from device memory (nitems_dev) and whose capacity sets
// the grid, so that a captured launch stays valid while solves join or
// leave; a list that outgrows its capacity needs a new capture.
hipError_t launch_stage_mfma_batch(int P, bool bf3, bool av, int waves, const void *jobs, const void *items,
                                   const int *nitems_dev, int capacity, hipStream_t st);
// CFL bound of state U (FP64) into the kVmaxSlots slots at *slot as bit
// patterns (the maximum over them is the bound); raises *flag on bad states.
// FP32 handles take the matrix-core kernel's own per-node bound
// (launch_cfl_vmax_mfma), so that a run's first step sees what a fused last
// stage would have left.
hipError_t launch_cfl_vmax(const DevMesh &m, const void *U, unsigned long long *slot, hipStream_t st);
hipError_t launch_cfl_vmax_mfma(const DevMesh &m, const void *U, unsigned long long *slots, hipStream_t st);
size_t mfma_opsA_floats(int P);
void mfma_fill_opsA(int P, const double *Dr, const double *Ds, const double *LIFT, float *out);
size_t mfma_opsB_words(int P);
void mfma_fill_opsB(int P, const double *Dr, const double *Ds, const double *LIFT, unsigned *out);
int mfma_elements_per_block(int P, int waves);
// setup: flags[k] = 1 if element k's metric terms, normals and Fscale are
// constant to 1e-10 relative (a straight element)
hipError_t launch_affine_flags(const DevMesh &m, int *flags, hipStream_t st);
// setup: pack the affine records of all elements and the per-node records
// of curved ones (cidx >= 0) from the FP64 tables
hipError_t launch_pack_geometry(const DevMesh &m, const int *cidx, float *geoA, float *geoC,
                                hipStream_t st);

// sensor: eps [K] (state precision) from U
hipError_t launch_sensor(const DevMesh &m, const void *U, void *eps, hipStream_t st);
// FP32 handles: the sensor plus the CFL bound of U with its new viscosity
// (FP32 per face node) reduced into the slots vmax[kVmaxSlots] (which must
// hold zeros or smaller bounds), and the state check into *flag
hipError_t launch_sensor_cfl(const DevMesh &m, const void *U, void *eps, unsigned long long *vmax,
                             hipStream_t st);
// LDG auxiliary gradient Q from U and eps
hipError_t launch_avgrad(const DevMesh &m, const void *U, const void *eps, void *Q, hipStream_t st);
// batched FP32 viscous handles of order P: per-(mesh, stage) argument
// records and the (record, tile) work list of the stage kernel's batch;
// one launch of the sensor (with the CFL bound when cfl) and one of the
// gradient over all of them
size_t av_args_bytes();
void av_fill_args(const DevMesh &m, const void *U, void *eps, void *Q, unsigned long long *vmax, void *out);
// items: (job, tile) pairs of the viscous kernels' tiles (av_tiles per
// mesh); eitems: (job, block) pairs of blocks of 256 elements for the
// per-element sensor
hipError_t launch_av_batch(int P, bool cfl, const void *jobs, const void *items, const int *nitems_dev,
                           int capacity, const void *eitems, const int *neitems_dev, int ecapacity,
                           hipStream_t st);
int sensor_elem_blocks(const DevMesh &m);
int av_tiles(const DevMesh &m);
// CFL reduction -> scal[S_DT] (dt_fixed > 0 overrides), accumulates S_T,
// S_DTMIN/MAX, S_STEPS; raises *flag on bad states.
hipError_t launch_cfl(const DevMesh &m, const void *U, const void *eps, double dt_fixed,
                      hipStream_t st);
// conserved totals -> scal[S_TOT..]
hipError_t launch_totals(const DevMesh &m, const void *U, hipStream_t st);
// max |rhs| per field -> scal[S_RES..]
hipError_t launch_residual(const DevMesh &m, const void *rhs, hipStream_t st);
// eps (state precision) -> double
hipError_t launch_eps_to_double(const DevMesh &m, const void *eps, double *out, hipStream_t st);
hipError_t launch_reset_scalars(const DevMesh &m, hipStream_t st);
// over-integrated weak form (weak.hip)
size_t weak_ops_size(int P);
hipError_t launch_weak_geometry(const DevMesh &m, const double *x, const double *y, const double *Drg,
                                const double *Dsg, const double *wg, double *geoA, double *geoF, double *geoC,
                                double *mass, double *work, hipStream_t st);
hipError_t launch_stage_weak(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                             hipStream_t st);
// the weak form on the matrix cores (weak_mfma.hip): FP32, every element straight
size_t weak_mfma_opsA_values(int P);
void weak_mfma_fill_opsA(int P, const double *Icub, const double *Drc, const double *Dsc, const double *If,
                         const double *Minv, float *out);
hipError_t launch_stage_weak_mfma(const DevMesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                                  hipStream_t st);
// p-refinement: U_to [K][4][np_to] = I (np_to x np_from, row-major, host) U_from
constexpr int kProlongMax = 21 * 21;
hipError_t launch_prolong(int K, int np_from, int np_to, const double *I, bool fp32, const void *Uf, void *Ut,
                          hipStream_t st);

// ---- 3D tetrahedra (tet3d.hip, api3.cpp)
struct Tet3Mesh {
    int K = 0, P = 0, Np = 0, Nfp = 0;
    bool fp32 = false;
    double gamma = 1.4, cfl = 0.5;
    const double *geo64 = nullptr;   // [K][25]
    const float *geo32 = nullptr;
    const float *opsA = nullptr;     // FP32 handles: matrix-core A operand (tet3_mfma_fill_opsA)
    const double *opsA64 = nullptr;  // FP64 handles: the same in FP64 (tet3_mfma_fill_opsA64)
    const int *fmap = nullptr;       // [K][4 Nfp]
    const int *fmask = nullptr;      // [4 Nfp]
    double *scal = nullptr;          // [S_NSCAL]
    unsigned long long *vmax = nullptr;   // [kSlots3] time-step bound slots
    int *flag = nullptr;
};
constexpr int kSlots3 = 64;   // one wavefront
int tet3_blocks(int K, int P);   // blocks of the time-step bound kernel
// A operand of the FP32 matrix-core stage [-Dr -Ds -Dt LIFT] in lane order
size_t tet3_mfma_opsA_values(int P);
void tet3_mfma_fill_opsA(int P, const double *Dr, const double *Ds, const double *Dt, const double *LIFT,
                         float *out);
void tet3_mfma_fill_opsA64(int P, const double *Dr, const double *Ds, const double *Dt, const double *LIFT,
                           double *out);
hipError_t launch_geometry3(int K, const double *X, double *geo, int *count, hipStream_t st);
// zeroes the scalars (dt_min = +inf), the bound and the flag
hipError_t launch_reset3(const Tet3Mesh &m, hipStream_t st);
// one stage (rhs != null: the bare rhs); bound: also the time-step bound of
// the new state into the slots and its state check (a step's last stage)
hipError_t launch_stage3(const Tet3Mesh &m, const void *Uin, void *Uout, void *R, void *rhs, int stage,
                         bool bound, hipStream_t st);
// time-step bound (FP64, from the state) into the slots; raises *flag on bad states
hipError_t launch_bound3(const Tet3Mesh &m, const void *U, hipStream_t st);
// dt = CFL / bound (dt_fixed > 0 overrides) into scal; clears the slots
hipError_t launch_dt3(const Tet3Mesh &m, double dt_fixed, hipStream_t st);
// error reporting shared with the 2D ABI (dg_last_error)
int report_error(int code, const std::string &msg);

}  // namespace dg
