/* C ABI of the 3D solver: nodal discontinuous Galerkin for the Euler
 * equations on straight tetrahedra, five conserved fields
 * (rho, rho u, rho v, rho w, E) -- the paper's own setting (Section 2, the
 * DG discretisation and the low-storage Runge-Kutta scheme; Section 5, the
 * 3D Euler system).  Shares the status codes, the precision enum, the run
 * statistics and dg_last_error with the 2D ABI in dg.h.
 *
 * Discretisation (the nodal strong form, as the 2D default):
 *   dU/dt = -(r_x Dr + s_x Ds + t_x Dt) F - (r_y Dr + ...) G - (r_z Dr + ...) H
 *           + LIFT (Fscale (n.F(U-) - F*))
 * with the local Lax-Friedrichs flux F* (Section 2, after eq. weak_dg),
 * the mirror ghost state at slip walls, and the Carpenter-Kennedy LSERK(5,4)
 * update.  Reference tetrahedron: vertices (-1,-1,-1), (1,-1,-1), (-1,1,-1),
 * (-1,-1,1); faces f0 = (v1 v2 v3), f1 = (v1 v2 v4), f2 = (v2 v3 v4),
 * f3 = (v1 v3 v4); nodes: the equispaced lattice (i, j, k) / P, r fastest,
 * then s, then t (Np = (P+1)(P+2)(P+3)/6, P = 1..4).
 *
 * Layouts: states are [K][5][Np] in the handle's precision (double for
 * DG_FP64_PLAIN, float for DG_FP32), on the device, 16-byte aligned (the
 * work buffer too); every array in dg3_mesh_desc is host memory, read
 * during dg3_mesh_setup only. */
#ifndef DG3_H
#define DG3_H

#include "dg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int K;                        /* elements, >= 1 */
    int P;                        /* order, 1..4 */
    int precision;                /* DG_FP64_PLAIN or DG_FP32 (both run the stage on the
                                     matrix cores, in FP64 and FP32 respectively) */
    const int *EToV;              /* [K][4] global vertex ids: faces match by their vertex triples */
    const int *EToE;              /* [K][4] neighbour across face f (the element itself at a wall) */
    const int *EToF;              /* [K][4] the neighbour's face */
    const signed char *bc;        /* [K][4] 0 interior, 1 slip wall (DG_BC_* of dg.h) */
    const double *X;              /* [K][4][3] vertex coordinates of each element, positively
                                     oriented (a periodic mesh gives each element its own image) */
    double gamma;                 /* ratio of specific heats, > 1 */
    double cfl;                   /* CFL number, > 0 */
} dg3_mesh_desc;

typedef struct dg3_mesh dg3_mesh;

/* Reference nodes (r, s, t arrays of Np doubles, caller-owned).
 * Errors: DG_EINVAL for P outside 1..4 or a NULL array. */
int dg3_reference_nodes(int P, double *r, double *s, double *t);

/* The reference operators of order P (host, FP64, caller-owned):
 * Dr, Ds, Dt [Np][Np] row-major (Dr = V_r V^-1 from a monomial basis,
 * each diagonal entry then set to minus the sum of its row's others, so that
 * rows sum to zero as the exact operator's do),
 * LIFT [Np][4 Nfp] (M^-1 E, exact simplex integrals; face f's block of Nfp
 * columns holds its face mass matrix), fmask [4][Nfp] the volume nodes of
 * each face in increasing order (f0: k = 0, f1: j = 0, f2: i + j + k = P,
 * f3: i = 0 on the lattice).  A NULL array is skipped.  No device work.
 * Errors: DG_EINVAL for P outside 1..4. */
int dg3_reference_operators(int P, double *Dr, double *Ds, double *Dt, double *LIFT, int *fmask);

/* Validates the desc as dg3_mesh_setup does and writes the neighbour node
 * map the solver uses (host int [K][4 Nfp], caller-owned):
 * fmap[k][f Nfp + j] = kn * 5 * Np + n, the offset in a [K][5][Np] state of
 * the neighbour's node n that coincides with face node j of face f (its
 * first field), or -1 at a wall.  No device work.
 * Errors: DG_EINVAL (bad mesh, with a message; K * 5 * Np beyond 2^31 - 1). */
int dg3_face_map(const dg3_mesh_desc *desc, int *fmap);

/* Validate the mesh (ids in range, reciprocal neighbours, matching face
 * vertex triples, walls where the desc says), build the operators (FP64 on
 * the host: Dr = V_r V^-1, ..., LIFT = M^-1 E from exact simplex
 * integrals), compute the geometric factors in FP64 on the device (metric
 * terms, outward unit normals, Fscale = (face area / 2) / (volume / (4/3))),
 * and the neighbour node map of every face node (by the barycentric lattice
 * indices of the face's shared vertices).  Enqueues on `stream` and
 * synchronises it.  *out receives the handle.
 * Errors: DG_EINVAL (bad mesh, with a message), DG_EGEOM (an element of
 * non-positive volume), DG_ENOMEM, DG_EDEVICE. */
int dg3_mesh_setup(const dg3_mesh_desc *desc, void *stream, dg3_mesh **out);

/* Frees the handle's device memory after the work it enqueued has ended. */
int dg3_mesh_destroy(dg3_mesh *mesh);

/* Bytes of one state array and of the work buffer dg3_run needs (the
 * Runge-Kutta register and two stage buffers, each starting on a 256-byte
 * boundary of the work buffer). */
int dg3_buffer_bytes(const dg3_mesh *mesh, size_t *state_bytes, size_t *work_bytes);

/* rhs = dU/dt of the device state U (no time stepping).  Enqueues only.
 * Errors: DG_EINVAL (NULL pointers, U == rhs, a pointer not 16-byte
 * aligned), DG_EDEVICE. */
int dg3_rhs(dg3_mesh *mesh, const void *U, void *rhs, void *stream);

/* nsteps LSERK steps of U in place, pairs of steps replayed from a graph
 * captured on the handle's own stream (built on the first call with these
 * U, work and dt_fixed, kept until they change).  dt_fixed > 0: that step; otherwise
 * dt = CFL / max over face nodes of (P+1)^2 Fscale (|v| + c) / 2, in FP64
 * from the state at the start of each step.  *stats (may be NULL) receives
 * steps, status, t, dt_min, dt_max and the device time (totals and
 * residual are zero in 3D).  Synchronises the stream.
 * Errors: DG_EINVAL, DG_ENONFINITE (non-finite state, rho <= 0 or p <= 0
 * at a face node), DG_EDEVICE. */
int dg3_run(dg3_mesh *mesh, void *U, void *work, int nsteps, double dt_fixed, dg_run_stats *stats,
            void *stream);

#ifdef __cplusplus
}
#endif

#endif
