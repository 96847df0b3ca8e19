/*
 * dg.h -- C ABI of the MI355X nodal discontinuous Galerkin solver for the 2D
 * Euler equations on unstructured, curved (isoparametric) triangles.
 *
 * What is computed (Siebenborn, Schulz, Schmidt, "A curved-element
 * unstructured discontinuous Galerkin method on GPUs for the Euler
 * equations"):
 *   dU/dt + div F(U) = 0 (Section 2, eq. conservation_law) discretised per
 *   element with a numerical flux on the element boundary (eq. weak_dg,
 *   local Lax-Friedrichs), mapped to the reference triangle through the
 *   metric terms of D Psi and J (Section 2), in the nodal strong form
 *       dU/dt = -(r_x Dr F + s_x Ds F + r_y Dr G + s_y Ds G)
 *               + LIFT [Fscale (n.F(U-) - F*)]
 *   (the semi-discrete system, eq. semidiscrete, with collocation at the
 *   nodes instead of cubature), optional Persson-Peraire artificial
 *   viscosity (Section 2: S_k, the eps_k ramp, q = sqrt(eps) grad U), and
 *   the low-storage 5-stage 4th-order Runge-Kutta scheme of Carpenter and
 *   Kennedy (Section 2).  The gas is perfect (Section 5) with 4 conserved
 *   fields (rho, rho u, rho v, E).
 *
 * Conventions
 *   - Reference triangle T = {r, s >= -1, r + s <= 0}, vertices
 *     v1=(-1,-1), v2=(1,-1), v3=(-1,1); faces 0: v1->v2, 1: v2->v3,
 *     2: v3->v1.  Elements must be counter-clockwise (J > 0).
 *   - Nodes per element Np = (P+1)(P+2)/2 in the order dg_reference_nodes
 *     returns; Nfp = P+1 nodes per face.
 *   - Neighbour face node of face node j is node Nfp-1-j of the
 *     neighbour's face (shared edges run in opposite directions).
 *   - State arrays are element-major [K][4][Np] in the handle's precision
 *     (double for DG_FP64_PLAIN, float for DG_FP32), on the device.
 *   - Boundary faces have EToE[k][f] = k, EToF[k][f] = f and a non-zero bc
 *     code; periodic seams are ordinary interior connectivity.
 *
 * Ownership: the caller owns every state and work buffer and the stream
 * (a hipStream_t passed as void*, NULL = the null stream); the handle owns
 * its device geometry and operator tables and frees them in
 * dg_mesh_destroy.  The library never frees caller memory.
 *
 * Errors: every function returns DG_OK (0) or a negative DG_E* code and
 * sets a thread-local message (dg_last_error).  No exceptions cross the ABI.
 * A handle is not thread-safe; different handles may run concurrently on
 * different streams.
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum dg_status {
    DG_OK = 0,
    DG_EINVAL = -1,      /* bad argument or inconsistent mesh */
    DG_ENOMEM = -2,      /* device allocation failed */
    DG_EGEOM = -3,       /* J <= 0 at some node, or mismatched face normals */
    DG_ENONFINITE = -4,  /* state became non-finite or rho <= 0 or p <= 0 */
    DG_EDEVICE = -5,     /* HIP runtime error */
    DG_EBUSY = -6        /* batch admission: no free slot, or over the HBM budget */
};

/* There is no separate DG_FP64 = 1: FP64 handles use DG_FP64_PLAIN, FP64
 * throughout.  Its stage runs on the VALUs, except for meshes whose elements
 * are all straight and carry no artificial viscosity, where the stage's
 * product runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64). */
enum dg_precision {
    DG_FP64_PLAIN = 0,   /* FP64 throughout */
    DG_FP32 = 2,         /* FP32 state and fused stage kernel; FP64 setup,
                            time step and reductions */
    DG_FP32_BF16X3 = 3   /* as DG_FP32, but the stage's matrix product runs as
                            three BF16 products of hi/lo splits,
                            A_hi B_hi + A_hi B_lo + A_lo B_hi, accumulated in
                            FP32 (about 16 significant bits per product;
                            fluxes, face terms and the update stay FP32) */
};

enum dg_bc { DG_BC_INTERIOR = 0, DG_BC_WALL = 1, DG_BC_FARFIELD = 2 };

/* Numerical flux at element faces (Section 2, after eq. weak_dg: local
 * Lax-Friedrichs, or HLLC, which the paper reports to behave alike).
 * HLLC: Davis wave-speed estimates and the star states of Toro, Spruce and
 * Speares, evaluated in the frame of the face normal. */
enum dg_riemann { DG_RIEMANN_LF = 0, DG_RIEMANN_HLLC = 1 };

/* Discretisation of the volume and surface terms.  DG_FORM_NODAL: the
 * nodal strong form (fluxes collocated at the nodes, Dr/Ds and LIFT).
 * DG_FORM_WEAK: the paper's over-integrated weak form (Section 2, eqs.
 * stiffness, mass, face_mass, semidiscrete): the state interpolated to a
 * collapsed Gauss product rule of n x n points exact for degree 3P
 * (n = (3P+2)/2) and to n Gauss points per face, M_k dU/dt = V - S with the
 * per-element mass matrix (inverted by Cholesky for curved elements at
 * setup).  Inviscid only (av_enable must be 0); FP64 or FP32 state, VALU
 * contractions; time step as for the nodal form. */
enum dg_form { DG_FORM_NODAL = 0, DG_FORM_WEAK = 1 };

/* Message of the last error on this thread ("" if none). */
const char *dg_last_error(void);

/* Library version (major*10000 + minor*100 + patch). */
int dg_version(void);

/* Reference nodes of order P (1 <= P <= 5): warp-and-blend nodes of
 * Warburton (2006), the family the paper cites for its collocation points
 * (Section 2), in rows of constant s (increasing s), increasing r within a
 * row.  r and s are host arrays of Np doubles, written by the call. */
int dg_reference_nodes(int P, double *r, double *s);

/* Face node ids (host int array of 3*Nfp): face f's nodes in
 * counter-clockwise traversal order. */
int dg_face_nodes(int P, int *fmask);

/* Reference operators of order P as built by the library (host, FP64,
 * row-major): Dr, Ds [Np*Np] (differentiation D_r = V_r V^{-1}, Section 2),
 * LIFT [Np*3*Nfp] (M^{-1} times the face mass matrix, the reference form of
 * M_k^{-1} M_dOmega in eq. semidiscrete), Vinv [Np*Np] (nodal to
 * orthonormal modal coefficients, f = V f_hat).  Any pointer may be NULL. */
int dg_reference_operators(int P, double *Dr, double *Ds, double *LIFT, double *Vinv);

/* Operators of the weak form of order P as built by the library (host,
 * FP64): *ncub cubature points and *ng Gauss points per face; wq [ncub]
 * weights, Icub, Drc, Dsc [ncub*Np] (nodal basis and its r, s derivatives
 * at the cubature points, row-major), wg [ng] face weights, If [ng*Nfp]
 * (the face nodes' 1D Lagrange basis at the face Gauss points).  Call with
 * NULL arrays to learn the sizes; any pointer may be NULL. */
int dg_weak_operators(int P, int *ncub, int *ng, double *wq, double *Icub, double *Drc, double *Dsc,
                      double *wg, double *If);

typedef struct {
    int K;                        /* elements, >= 1 */
    int P;                        /* order, 1..5 */
    int precision;                /* enum dg_precision */
    double gamma;                 /* ratio of specific heats, > 1 */
    double cfl;                   /* CFL number of the automatic step, > 0 */
    const int *EToE;              /* host [K][3] neighbour element */
    const int *EToF;              /* host [K][3] neighbour face */
    const signed char *bc;        /* host [K][3] enum dg_bc */
    const double *x, *y;          /* host [K][Np] node coordinates (curved) */
    double freestream[4];         /* far-field state (rho, rho u, rho v, E) */
    int av_enable;                /* Persson-Peraire artificial viscosity */
    double av_eps0;               /* eps_max = av_eps0 * h_k / P */
    double av_s0;                 /* ramp centre; NaN: -4 log10 P */
    double av_kappa;              /* ramp half-width, > 0 */
    int riemann;                  /* enum dg_riemann */
    int form;                     /* enum dg_form */
} dg_mesh_desc;

typedef struct dg_mesh dg_mesh;   /* opaque handle */

typedef struct {
    int steps;                    /* steps taken by the call */
    int status;                   /* DG_OK or DG_ENONFINITE */
    double t;                     /* simulated time advanced by the call */
    double dt_min, dt_max;        /* time steps used */
    double totals[4];             /* conserved totals at the end (FP64) */
    double residual[4];           /* ||dU/dt||_inf per field at the end */
    double wall_s;                /* device time of the call (HIP events) */
    double dof_updates_per_s;     /* 4*Np*K*5*steps / wall_s */
} dg_run_stats;

/* Validate the mesh, build operators, upload connectivity and compute the
 * geometric factors in FP64 on the device (metric terms of the
 * isoparametric map per node, Section 2; face normals, sJ, Fscale per face
 * node).  Checks: 1 <= P <= 5, K >= 1, reciprocal connectivity
 * (EToE[EToE[k][f]][EToF[k][f]] = k), valid bc codes, J > 0 at every node
 * (else DG_EGEOM), n- = -n+ within 1e-10 at interior face nodes (else
 * DG_EGEOM).  Viscous handles also allocate here the scratch of dg_rhs and
 * dg_viscosity, so that those calls allocate nothing.  Synchronises the
 * stream.  *out is NULL on error. */
int dg_mesh_setup(const dg_mesh_desc *desc, void *stream, dg_mesh **out);

/* Wait for the work the handle's last call enqueued (on the stream it was
 * given; work the caller enqueued elsewhere is not waited for), then free
 * the handle's device tables. */
int dg_mesh_destroy(dg_mesh *mesh);

/* Bytes of one state array [K][4][Np] and of the work buffer that
 * dg_step/dg_run need. */
int dg_buffer_bytes(const dg_mesh *mesh, size_t *state_bytes, size_t *work_bytes);

/* rhs = dU/dt for state U (device pointers, [K][4][Np]).  t is accepted for
 * interface completeness; the boundary data are time-independent.
 * Enqueues only (no allocation; may be captured into a graph).  Viscous
 * handles use the handle's own scratch, so two dg_rhs calls on one handle
 * must not overlap on different streams. */
int dg_rhs(dg_mesh *mesh, const void *U, void *rhs, double t, void *stream);

/* One LSERK(5,4) step of U in place.  dt > 0: that step; dt <= 0: the CFL
 * step computed on the device from U (dt = cfl / max over face nodes of
 * (P+1)^2/2 Fscale (|v|+c) + (P+1)^4/4 Fscale^2 eps).  work: device buffer
 * of dg_buffer_bytes' work_bytes.  Enqueues only (no host round trip). */
int dg_step(dg_mesh *mesh, void *U, void *work, double dt, void *stream);

/* Size of the static work area of dg_step_static (256 MiB). */
#define DG_STATIC_WORK_BYTES (256u << 20)

/* dg_step without a work argument, for callers that cannot allocate device
 * memory (code under stream capture, serving loops, harnesses that forbid
 * allocation): the work buffer is a file-scope device array of
 * DG_STATIC_WORK_BYTES that every GPU the library runs on holds until the
 * process ends.  The call allocates nothing.  Meshes whose work_bytes
 * (dg_buffer_bytes) exceed DG_STATIC_WORK_BYTES get DG_EINVAL.  Nothing in
 * the area needs to start at zero: a step writes the Runge-Kutta register
 * and the stage buffers before it reads them.  All calls on one GPU share
 * the area: calls that overlap on one GPU (different streams, or different
 * handles at once) race.  Same results as dg_step with a caller work buffer.
 * Enqueues only. */
int dg_step_static(dg_mesh *mesh, void *U, double dt, void *stream);

/* nsteps CFL steps of U in place, then totals and residual; synchronises
 * and fills *stats (may be NULL).  Returns DG_ENONFINITE if the state
 * became non-finite, rho <= 0 or p <= 0 at any step.  FP32 handles take
 * the CFL bound from the stage kernels themselves (without viscosity: the
 * last stage, for the next step, and a kernel with the same per-node
 * arithmetic before the first step; with viscosity: the first stage's
 * sensor), evaluated in FP64 per node from the FP32 state; FP64 handles
 * and dg_step use the FP64 reduction.  Calls compose: dg_run of N steps
 * twice gives the same bits as one dg_run of 2N steps. */
int dg_run(dg_mesh *mesh, void *U, void *work, int nsteps, dg_run_stats *stats, void *stream);

/* Conserved totals sum_k sum_i w_ki U_ki, w_ki = sum_j M_ij J_kj, in FP64
 * (host out[4]).  Synchronises. */
int dg_totals(dg_mesh *mesh, const void *U, double out[4], void *stream);

/* Residual ||rhs(U)||_inf per field (host out[4]), the convergence monitor
 * of the paper (Section 5).  work as for dg_step.  Synchronises. */
int dg_residual(dg_mesh *mesh, const void *U, void *work, double out[4], void *stream);

/* Element viscosities eps_k of state U (device out [K] doubles).  Enqueues
 * only (FP32 handles use scratch allocated at setup).  Returns DG_EINVAL if
 * the mesh was set up without viscosity. */
int dg_viscosity(dg_mesh *mesh, const void *U, double *eps, void *stream);

/* p-refinement (Section 5, the p-refinement paragraph): the prolongation
 * operator from order P to order Q >= P (host, row-major Np(Q) x Np(P)),
 * I = V_Q[:, :Np(P)] V_P^{-1}: the degree-P polynomial evaluated at the
 * order-Q nodes, which is the zero padding of its hierarchical modal
 * coefficients (the first Np(P) modes of order Q's basis span degree <= P). */
int dg_prolong_operator(int P, int Q, double *I);

/* U_to = I U_from per element and field, from the state of handle `from`
 * (order P) to that of handle `to` (order Q >= P); the two handles must
 * describe the same elements (same K, same precision).  Device pointers
 * [K][4][Np(P)] and [K][4][Np(Q)].  Enqueues only. */
int dg_prolong(const dg_mesh *from, const void *U_from, const dg_mesh *to, void *U_to, void *stream);

/* Replay of captured steps.  With graphs enabled (the default), dg_run on
 * an FP32 handle (with or without artificial viscosity) captures two steps
 * into a hipGraph once per (U, work) pair and replays it, which removes
 * per-launch host overhead; the arithmetic is identical to the eager
 * launches.  Graphs are not used while kernel timing is enabled. */
int dg_set_graphs(dg_mesh *mesh, int enable);

/* Per-launch timing of the fused stage kernel.  With timing enabled,
 * dg_step and dg_run bracket every stage-kernel launch with a pair of HIP
 * events on the caller's stream (no synchronisation).  dg_kernel_time
 * synchronises the stream, adds up the elapsed times of all bracketed
 * launches since the last call, returns the total in milliseconds and the
 * number of launches, and resets both.  Used by benchmarks to report the
 * dominant kernel's average duration measured inside the timed region. */
int dg_set_kernel_timing(dg_mesh *mesh, int enable);

/* Autotuner for the workgroup shape of the FP32 matrix-core stage kernel:
 * elements per workgroup = 2, 4 or 8 wavefronts times the elements one
 * wavefront holds (floor(64 / Np)).  The shape is a launch parameter, not
 * part of the method: results do not depend on it.
 * If the process tuning table (below) holds a shape for this handle's kind
 * (device architecture, P, precision, viscosity), applies it and returns it
 * with *stage_us = 0 without timing.  Otherwise times each candidate over
 * Runge-Kutta stage evaluations of the device state U [K][4][Np] (written
 * into the work buffer, whose contents between steps are scratch; U is only
 * read; a viscous handle's viscosity and sigma grad U of U are computed
 * there first), keeps the fastest for this handle and records it in the
 * table.  *waves_per_block receives the choice and *stage_us the measured
 * time of one launch (either may be NULL).  FP64 and weak-form handles have
 * no shape to tune and return DG_OK with 0.
 * Synchronises the stream.  Errors: DG_EINVAL, DG_EDEVICE. */
int dg_autotune(dg_mesh *mesh, const void *U, void *work, void *stream, int *waves_per_block,
                double *stage_us);
int dg_kernel_time(dg_mesh *mesh, void *stream, double *stage_ms_total, long *stage_launches);

/* Tuning table: one workgroup shape (waves per workgroup: 2, 4 or 8) per
 * (device architecture name such as "gfx950", P, precision DG_FP32 or
 * DG_FP32_BF16X3, av_enable 0/1), process-wide and thread-safe.  A new
 * handle takes its kind's entry (unless the environment variable
 * DG_WAVES_PER_BLOCK sets the shape); a batch takes it for a kind of solve
 * when that kind first joins the batch and keeps it for the batch's life.
 * dg_autotune fills it; dg_tuning_save/dg_tuning_load persist it as text,
 * one entry per line: "arch P precision av waves stage_us" ('#' starts a
 * comment line); a load merges into the table and rejects the whole file
 * (DG_EINVAL, naming the line) if any entry is malformed.  *entries (may be
 * NULL) receives the number of entries written or read.  dg_tuning_lookup
 * gives 0 for a kind with no entry; dg_device_arch writes the current
 * device's architecture name (NUL-terminated; DG_EINVAL if size is too
 * small).  Errors: DG_EINVAL. */
int dg_tuning_set(const char *arch, int P, int precision, int av_enable, int waves_per_block);
int dg_tuning_lookup(const char *arch, int P, int precision, int av_enable, int *waves_per_block);
int dg_tuning_clear(void);
int dg_tuning_save(const char *path, int *entries);
int dg_tuning_load(const char *path, int *entries);
int dg_device_arch(char *buf, size_t size);

/* Device bytes a handle holds (geometry, operators, scratch) plus one state
 * array and its work buffer: the unit of HBM-footprint admission. */
int dg_mesh_footprint(const dg_mesh *mesh, size_t *bytes);

/* Number of elements the handle treats as curved: those whose metric terms
 * vary over the element beyond rounding (relative 1e-10 of the element's
 * largest metric term) or whose face normals and Fscale vary along a face
 * (Section 2, the isoparametric map; an affine element's map has constant
 * metric terms).  Curved elements keep per-node (nodal form) or
 * per-cubature-point (weak form) metric terms and, in the weak form, their
 * own inverse mass matrix; the others use five to thirteen numbers.  -1 for
 * FP64 nodal handles, whose stage kernel takes per-node metrics for every
 * element.  Errors: DG_EINVAL. */
int dg_mesh_curved(const dg_mesh *mesh, int *curved);

/* Upper estimate of dg_mesh_footprint for a mesh not yet set up, so that a
 * server can decide admission before allocating anything. */
int dg_estimate_footprint(int K, int P, int precision, int av_enable, size_t *bytes);

/* ---- Batching (continuous batching of independent solves) ----------------
 * A batch holds up to max_slots independent solves (each a dg_mesh with its
 * own state U and work buffer, all on one device) whose summed footprints
 * stay within hbm_budget_bytes.  dg_batch_advance moves every active slot
 * forward in lockstep: for each order P, precision mode and viscosity
 * setting one launch per RK stage covers the tiles of all FP32 slots of
 * that kind (viscous slots add one sensor and one gradient launch per
 * stage over all of them), each with its own CFL time step computed on the
 * device; FP64 slots are stepped one by one in the same stream.  Two steps are captured in a hipGraph and replayed
 * (see dg_batch_info for when it is captured again).  The result of every slot is
 * bit-identical to running it alone with dg_run.  Slots join (admit) and
 * leave (release) between calls, so solves that arrive while others are
 * running start at the next call. */
typedef struct dg_batch dg_batch;

/* A batch takes handles of any precision (each handle's own); there is no
 * per-batch precision argument. */
int dg_batch_create(size_t hbm_budget_bytes, int max_slots, dg_batch **out);
/* Waits for the batch's last advance, then frees its tables. */
int dg_batch_destroy(dg_batch *batch);

/* Admit a solve of nsteps CFL steps.  DG_EBUSY if no slot is free or the
 * footprint does not fit the budget (the caller keeps it queued).  Resets
 * the handle's time and statistics.  Enqueues on stream. */
int dg_batch_admit(dg_batch *batch, dg_mesh *mesh, void *U, void *work, int nsteps, void *stream,
                   int *slot);

/* Advance all active slots by min(max_steps, fewest remaining steps) steps;
 * *steps_run receives that number.  Enqueues only. */
int dg_batch_advance(dg_batch *batch, int max_steps, void *stream, int *steps_run);

/* Synchronise the stream and list slots that are done and not yet released
 * (up to max_done ids; *ndone = how many).  A slot is done when it has run
 * all its steps, or when its state check has failed (non-finite state,
 * rho <= 0 or p <= 0): such a slot retires at this poll, and its stats
 * report DG_ENONFINITE and the steps it ran. */
int dg_batch_poll(dg_batch *batch, void *stream, int *done_slots, int max_done, int *ndone);

/* Steps done, simulated time, dt range and status of a slot (synchronises). */
int dg_batch_slot_stats(dg_batch *batch, int slot, void *stream, dg_run_stats *stats);

/* Step graphs the batch has captured so far, and the kinds of solve (order,
 * product precision, viscosity) it holds tables for.  The batched launches
 * read their work lists' lengths from device memory and a kind's tables
 * stay once created, so the captured two-step graph stays valid while
 * solves join and leave; it is captured again only when a new kind
 * appears, a work list outgrows its table or the set of FP64 slots (stepped
 * one by one inside the graph) changes. */
int dg_batch_info(dg_batch *batch, int *captures, int *groups);

/* Free a slot and its share of the budget; the handle and buffers stay the
 * caller's. */
int dg_batch_release(dg_batch *batch, int slot);

/* Device flag of the last dg_step/dg_run: 1 if a non-finite state,
 * rho <= 0 or p <= 0 was seen.  Synchronises the stream. */
int dg_status(dg_mesh *mesh, void *stream, int *device_flag);

#ifdef __cplusplus
}
#endif

#endif /* DG_H */
