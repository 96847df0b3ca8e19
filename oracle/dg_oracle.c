/*
 * Plain FP64 CPU oracle for the nodal DG discretisation of the 2D Euler
 * equations on curved triangles, with the Persson-Peraire sensor, LDG
 * artificial viscosity and the 5-stage 4th-order low-storage Runge-Kutta
 * scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library; the solver never
 * links or calls it, and it shares no source with the solver.
 *
 * It is written for readability: one element at a time, plain loops, no
 * blocking or fusion beyond what the equations state, reductions in serial
 * order.  OpenMP only distributes the independent per-element loops.
 *
 * Paper sections followed (Siebenborn, Schulz, Schmidt, "A curved-element
 * unstructured discontinuous Galerkin method on GPUs for the Euler
 * equations"):
 *   - conservation law and the weak DG form with a numerical flux
 *     (Section 2, eqs. conservation_law and weak_dg), here in the
 *     equivalent strong nodal form with reference differentiation and LIFT;
 *   - the reference map and its metric terms r_x, ... and J (Section 2, the
 *     D Psi matrix), evaluated per node for curved elements;
 *   - the local Lax-Friedrichs flux (Section 2, after eq. weak_dg);
 *   - the semi-discrete system (eq. semidiscrete) and the low-storage RK
 *     scheme of Carpenter and Kennedy (Section 2);
 *   - the smoothness indicator S_k, s_k = log10 S_k and the sine ramp for
 *     eps_k, and the first-order viscous system q = sqrt(eps) grad U
 *     (Section 2, artificial viscosity);
 *   - the 3D Euler system and the perfect-gas law (Section 5), reduced to
 *     2D with E the total energy density;
 *   - the residual infinity norm used as the convergence monitor (Section 5).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NF 4 /* conserved fields: rho, rho u, rho v, E */

enum { BC_INTERIOR = 0, BC_WALL = 1, BC_FARFIELD = 2 };

/* Cubature operators of the over-integrated weak form (Section 2, eqs.
 * stiffness, mass, face_mass, semidiscrete): a rule of ncub points on the
 * reference triangle and ng Gauss points per face. */
typedef struct {
    int ncub, ng;
    const double *wq;        /* [ncub] cubature weights (sum 2) */
    const double *Icub;      /* [ncub][Np] nodal basis at the cubature points */
    const double *Drc, *Dsc; /* [ncub][Np] its r and s derivatives there */
    const double *wg;        /* [ng] Gauss weights on [-1, 1] */
    const double *If;        /* [ng][Nfp] face-node Lagrange basis at the Gauss points */
    const double *Drg, *Dsg; /* [3][ng][Np] basis derivatives at each face's Gauss points */
} oracle_weak;

typedef struct {
    int K, P, Np, Nfp;
    double gamma;
    /* reference operators, row-major */
    const double *Dr, *Ds;   /* [Np][Np] */
    const double *LIFT;      /* [Np][3*Nfp] */
    const double *Vinv;      /* [Np][Np]: modal = Vinv * nodal */
    const double *Mref;      /* [Np][Np] */
    const int *Fmask;        /* [3][Nfp], CCW per face */
    const int *top_modes;    /* [Nfp] modal indices of total degree P */
    /* connectivity */
    const int *EToE, *EToF;  /* [K][3] */
    const signed char *bc;   /* [K][3] */
    /* geometric factors (oracle_geometry fills them) */
    const double *rx, *sx, *ry, *sy, *J; /* [K][Np] */
    const double *nx, *ny, *Fscale;      /* [K][3*Nfp] */
    double freestream[NF];
    double cfl;
    int av_enable;
    double av_eps0, av_s0, av_kappa;
    int riemann;          /* numerical flux: 0 local Lax-Friedrichs, 1 HLLC */
    /* test switches */
    int no_euler_flux;    /* 1: drop the inviscid flux (pure diffusion tests) */
    double eps_override;  /* >= 0: this viscosity in every element */
    /* scratch owned by the caller: [K] eps, [K][2][NF][Np] Q */
    double *eps, *Q;
    /* over-integrated weak form (NULL: the nodal strong form) with the
     * element node coordinates it needs for its metric terms */
    const oracle_weak *weak;
    const double *x, *y;     /* [K][Np] */
} oracle_mesh;

/* ---------------------------------------------------------------------- */
/* pointwise gas dynamics                                                 */
/* ---------------------------------------------------------------------- */

static double pressure(double g, const double u[NF]) {
    /* perfect gas: p = (gamma-1)(E - (m_x^2 + m_y^2)/(2 rho)) */
    return (g - 1.0) * (u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) / u[0]);
}

static void euler_flux(double g, const double u[NF], double F[NF], double G[NF]) {
    double rho = u[0], mx = u[1], my = u[2], E = u[3];
    double p = pressure(g, u);
    F[0] = mx;
    F[1] = mx * mx / rho + p;
    F[2] = mx * my / rho;
    F[3] = (E + p) * mx / rho;
    G[0] = my;
    G[1] = mx * my / rho;
    G[2] = my * my / rho + p;
    G[3] = (E + p) * my / rho;
}

/* Normal flux n.F(u) and the wave speed |v.n| + c. */
static void normal_flux(double g, const double u[NF], double nx, double ny,
                        double fn[NF], double *lam) {
    double F[NF], G[NF];
    euler_flux(g, u, F, G);
    for (int c = 0; c < NF; ++c) fn[c] = nx * F[c] + ny * G[c];
    double vn = (u[1] * nx + u[2] * ny) / u[0];
    double cs = sqrt(g * pressure(g, u) / u[0]);
    *lam = fabs(vn) + cs;
}

/* Local Lax-Friedrichs flux F* = 1/2 (n.F(u-) + n.F(u+)) - 1/2 lam (u+ - u-),
 * with lam the larger of the two local wave speeds at this face node. */
void oracle_lf_flux(double g, const double um[NF], const double up[NF],
                    double nx, double ny, double fstar[NF]) {
    double fm[NF], fp[NF], lm, lp;
    normal_flux(g, um, nx, ny, fm, &lm);
    normal_flux(g, up, nx, ny, fp, &lp);
    double lam = lm > lp ? lm : lp;
    for (int c = 0; c < NF; ++c)
        fstar[c] = 0.5 * (fm[c] + fp[c]) - 0.5 * lam * (up[c] - um[c]);
}

/* HLLC flux (Toro, Spruce and Speares; Toro's book, chapter 10) in the
 * frame of the face normal n, a selectable alternative to the local
 * Lax-Friedrichs flux (the paper reports both, Section 2 after eq. weak_dg).
 * Wave speeds: S_L = min(v_n- - c-, v_n+ - c+), S_R = max(v_n- + c-,
 * v_n+ + c+) (Davis); contact speed
 *   S* = (p+ - p- + rho- v_n- (S_L - v_n-) - rho+ v_n+ (S_R - v_n+))
 *        / (rho- (S_L - v_n-) - rho+ (S_R - v_n+)).
 * Star state of side K (velocity v_K + (S* - v_nK) n, i.e. the normal
 * velocity replaced by S*):
 *   U*_K = rho_K (S_K - v_nK)/(S_K - S*) (1, v_K + (S* - v_nK) n,
 *          E_K/rho_K + (S* - v_nK)(S* + p_K/(rho_K (S_K - v_nK)))).
 * F* = n.F(U-) if S_L >= 0; n.F(U-) + S_L (U*_L - U-) if S_L < 0 <= S*;
 * n.F(U+) + S_R (U*_R - U+) if S* < 0 < S_R; n.F(U+) if S_R <= 0. */
static void hllc_star(double g, const double u[NF], double nx, double ny, double SK, double Ss,
                      double out[NF]) {
    double rho = u[0], vx = u[1] / rho, vy = u[2] / rho;
    double p = pressure(g, u);
    double vn = vx * nx + vy * ny;
    double f = rho * (SK - vn) / (SK - Ss);
    out[0] = f;
    out[1] = f * (vx + (Ss - vn) * nx);
    out[2] = f * (vy + (Ss - vn) * ny);
    out[3] = f * (u[3] / rho + (Ss - vn) * (Ss + p / (rho * (SK - vn))));
}

void oracle_hllc_flux(double g, const double um[NF], const double up[NF],
                      double nx, double ny, double fstar[NF]) {
    double fm[NF], fp[NF], lm, lp;
    normal_flux(g, um, nx, ny, fm, &lm);
    normal_flux(g, up, nx, ny, fp, &lp);
    double rl = um[0], rr = up[0];
    double vnl = (um[1] * nx + um[2] * ny) / rl, vnr = (up[1] * nx + up[2] * ny) / rr;
    double pl = pressure(g, um), pr = pressure(g, up);
    double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
    double SL = fmin(vnl - cl, vnr - cr);
    double SR = fmax(vnl + cl, vnr + cr);
    double Ss = (pr - pl + rl * vnl * (SL - vnl) - rr * vnr * (SR - vnr)) /
                (rl * (SL - vnl) - rr * (SR - vnr));
    if (SL >= 0.0) {
        for (int c = 0; c < NF; ++c) fstar[c] = fm[c];
    } else if (Ss >= 0.0) {
        double us[NF];
        hllc_star(g, um, nx, ny, SL, Ss, us);
        for (int c = 0; c < NF; ++c) fstar[c] = fm[c] + SL * (us[c] - um[c]);
    } else if (SR > 0.0) {
        double us[NF];
        hllc_star(g, up, nx, ny, SR, Ss, us);
        for (int c = 0; c < NF; ++c) fstar[c] = fp[c] + SR * (us[c] - up[c]);
    } else {
        for (int c = 0; c < NF; ++c) fstar[c] = fp[c];
    }
}

/* Ghost state of a boundary face node (outward unit normal n).
 * Slip wall: mirror the momentum, u+ = (rho, m - 2 (m.n) n, E).
 * Far field: characteristic state from the Riemann invariants
 *   R_out = v_n + 2c/(g-1) (interior), R_in = v_n,inf - 2c_inf/(g-1),
 * entropy and tangential velocity from the upwind side; supersonic inflow
 * takes the free stream, supersonic outflow the interior state. */
void oracle_ghost(double g, int code, const double um[NF], double nx, double ny,
                  const double qinf[NF], double up[NF]) {
    if (code == BC_WALL) {
        double mn = um[1] * nx + um[2] * ny;
        up[0] = um[0];
        up[1] = um[1] - 2.0 * mn * nx;
        up[2] = um[2] - 2.0 * mn * ny;
        up[3] = um[3];
        return;
    }
    /* far field */
    double rhoi = um[0], ui = um[1] / rhoi, vi = um[2] / rhoi;
    double pi = pressure(g, um), ci = sqrt(g * pi / rhoi);
    double vni = ui * nx + vi * ny;
    double rhoo = qinf[0], uo = qinf[1] / rhoo, vo = qinf[2] / rhoo;
    double po = pressure(g, qinf), co = sqrt(g * po / rhoo);
    double vno = uo * nx + vo * ny;
    if (vni <= -ci) { /* supersonic inflow */
        for (int c = 0; c < NF; ++c) up[c] = qinf[c];
        return;
    }
    if (vni >= ci) { /* supersonic outflow */
        for (int c = 0; c < NF; ++c) up[c] = um[c];
        return;
    }
    double Rout = vni + 2.0 * ci / (g - 1.0);
    double Rin = vno - 2.0 * co / (g - 1.0);
    double vnb = 0.5 * (Rout + Rin);
    double cb = 0.25 * (g - 1.0) * (Rout - Rin);
    double sb, utb, vtb;
    if (vnb > 0.0) { /* outflow: entropy and tangential velocity from inside */
        sb = pi / pow(rhoi, g);
        utb = ui - vni * nx;
        vtb = vi - vni * ny;
    } else {
        sb = po / pow(rhoo, g);
        utb = uo - vno * nx;
        vtb = vo - vno * ny;
    }
    double rhob = pow(cb * cb / (g * sb), 1.0 / (g - 1.0));
    double pb = rhob * cb * cb / g;
    double ub = utb + vnb * nx, vb = vtb + vnb * ny;
    up[0] = rhob;
    up[1] = rhob * ub;
    up[2] = rhob * vb;
    up[3] = pb / (g - 1.0) + 0.5 * rhob * (ub * ub + vb * vb);
}

/* ---------------------------------------------------------------------- */
/* geometry                                                               */
/* ---------------------------------------------------------------------- */

/* Per-node metric terms of the isoparametric map (x, y nodal coordinates):
 * x_r = Dr x, ..., J = x_r y_s - x_s y_r, r_x = y_s/J, s_x = -y_r/J,
 * r_y = -x_s/J, s_y = x_r/J.  Per face node: outward normal from the same
 * metrics (face 0: (y_r, -x_r), face 1: (y_s - y_r, x_r - x_s),
 * face 2: (-y_s, x_s)), sJ its length, n = ./sJ, Fscale = sJ/J.
 * Returns the number of nodes with J <= 0. */
long oracle_geometry(const oracle_mesh *m, const double *x, const double *y,
                     double *rx, double *sx, double *ry, double *sy, double *J,
                     double *nx, double *ny, double *sJ, double *Fscale) {
    const int Np = m->Np, Nfp = m->Nfp;
    long bad = 0;
#pragma omp parallel for reduction(+ : bad)
    for (long k = 0; k < m->K; ++k) {
        const double *xk = x + k * Np, *yk = y + k * Np;
        double xr[64], xs[64], yr[64], ys[64];
        for (int i = 0; i < Np; ++i) {
            double a = 0, b = 0, c = 0, d = 0;
            for (int j = 0; j < Np; ++j) {
                a += m->Dr[i * Np + j] * xk[j];
                b += m->Ds[i * Np + j] * xk[j];
                c += m->Dr[i * Np + j] * yk[j];
                d += m->Ds[i * Np + j] * yk[j];
            }
            xr[i] = a; xs[i] = b; yr[i] = c; ys[i] = d;
            double jac = a * d - b * c;
            if (!(jac > 0.0)) bad++;
            J[k * Np + i] = jac;
            rx[k * Np + i] = d / jac;
            sx[k * Np + i] = -c / jac;
            ry[k * Np + i] = -b / jac;
            sy[k * Np + i] = a / jac;
        }
        for (int f = 0; f < 3; ++f)
            for (int j = 0; j < Nfp; ++j) {
                int v = m->Fmask[f * Nfp + j];
                double ax, ay;
                if (f == 0) { ax = yr[v]; ay = -xr[v]; }
                else if (f == 1) { ax = ys[v] - yr[v]; ay = xr[v] - xs[v]; }
                else { ax = -ys[v]; ay = xs[v]; }
                double len = sqrt(ax * ax + ay * ay);
                long q = k * 3 * Nfp + f * Nfp + j;
                nx[q] = ax / len;
                ny[q] = ay / len;
                sJ[q] = len;
                Fscale[q] = len / J[k * Np + v];
            }
    }
    return bad;
}

/* ---------------------------------------------------------------------- */
/* sensor and artificial viscosity                                        */
/* ---------------------------------------------------------------------- */

/* Persson-Peraire smoothness indicator of the density: modal coefficients
 * u_hat = V^{-1} rho; S_k = (energy in the degree-P modes) / (total energy),
 * both in the orthonormal basis (reference-element L2 norms);
 * s_k = log10 S_k and the sine ramp around s0 of half-width kappa, capped at
 * eps_max = eps0 * h_k / P with h_k = 2 / max Fscale. */
double oracle_sensor_element(const oracle_mesh *m, long k, const double *U) {
    const int Np = m->Np, Nfp = m->Nfp;
    const double *rho = U + k * NF * Np; /* field 0 */
    double num = 0.0, den = 0.0;
    for (int n = 0; n < Np; ++n) {
        double uh = 0.0;
        for (int j = 0; j < Np; ++j) uh += m->Vinv[n * Np + j] * rho[j];
        den += uh * uh;
        int top = 0;
        for (int t = 0; t < Nfp; ++t) top |= (m->top_modes[t] == n);
        if (top) num += uh * uh;
    }
    double fmax = 0.0;
    for (int q = 0; q < 3 * Nfp; ++q) {
        double fs = m->Fscale[k * 3 * Nfp + q];
        if (fs > fmax) fmax = fs;
    }
    double h = 2.0 / fmax;
    double emax = m->av_eps0 * h / m->P;
    if (!(den > 1e-300) || !(num > 0.0)) return 0.0;
    double sk = log10(num / den);
    double s0 = m->av_s0, kap = m->av_kappa;
    if (sk < s0 - kap) return 0.0;
    if (sk > s0 + kap) return emax;
    return 0.5 * emax * (1.0 + sin(M_PI * (sk - s0) / (2.0 * kap)));
}

void oracle_sensor(const oracle_mesh *m, const double *U, double *eps) {
#pragma omp parallel for
    for (long k = 0; k < m->K; ++k) eps[k] = oracle_sensor_element(m, k, U);
}

static double elem_eps(const oracle_mesh *m, const double *U, long k) {
    if (m->eps_override >= 0.0) return m->eps_override;
    return oracle_sensor_element(m, k, U);
}

/* Trace value of element k, face f, face node j, and the state across it:
 * the neighbour's node Nfp-1-j on its face (shared edges are traversed in
 * opposite directions), or the boundary ghost state. */
static void face_states(const oracle_mesh *m, const double *U, long k, int f, int j,
                        double um[NF], double up[NF], long *kn_out, int *vn_out) {
    const int Np = m->Np, Nfp = m->Nfp;
    int v = m->Fmask[f * Nfp + j];
    for (int c = 0; c < NF; ++c) um[c] = U[(k * NF + c) * Np + v];
    int code = m->bc[k * 3 + f];
    long q = k * 3 * Nfp + f * Nfp + j;
    if (code == BC_INTERIOR) {
        long kn = m->EToE[k * 3 + f];
        int fn = m->EToF[k * 3 + f];
        int vn = m->Fmask[fn * Nfp + (Nfp - 1 - j)];
        for (int c = 0; c < NF; ++c) up[c] = U[(kn * NF + c) * Np + vn];
        *kn_out = kn;
        *vn_out = vn;
    } else {
        oracle_ghost(m->gamma, code, um, m->nx[q], m->ny[q], m->freestream, up);
        *kn_out = -1;
        *vn_out = -1;
    }
}

/* Auxiliary variable of the first-order viscous system, q = sigma grad U with
 * sigma = sqrt(eps_k), in strong DG form with the central trace
 * (sigma U)* = 1/2 (sigma- U- + sigma+ U+) (boundary: sigma- (U- + U_ghost)/2):
 *   Q_x = sigma (r_x Dr U + s_x Ds U) + LIFT [Fscale n_x ((sigma U)* - sigma U-)]
 * and likewise Q_y.  Q layout [K][2][NF][Np]. */
void oracle_av_gradient(const oracle_mesh *m, const double *U, const double *eps,
                        double *Q) {
    const int Np = m->Np, Nfp = m->Nfp, Nf3 = 3 * m->Nfp;
#pragma omp parallel for
    for (long k = 0; k < m->K; ++k) {
        double sig = sqrt(eps[k]);
        double jx[3 * 16][NF], jy[3 * 16][NF];
        for (int f = 0; f < 3; ++f)
            for (int j = 0; j < Nfp; ++j) {
                double um[NF], up[NF];
                long kn;
                int vn;
                face_states(m, U, k, f, j, um, up, &kn, &vn);
                double sigp = (kn >= 0) ? sqrt(eps[kn]) : sig;
                long q = k * Nf3 + f * Nfp + j;
                for (int c = 0; c < NF; ++c) {
                    double star = 0.5 * (sig * um[c] + sigp * up[c]);
                    double d = m->Fscale[q] * (star - sig * um[c]);
                    jx[f * Nfp + j][c] = m->nx[q] * d;
                    jy[f * Nfp + j][c] = m->ny[q] * d;
                }
            }
        for (int c = 0; c < NF; ++c) {
            const double *u = U + (k * NF + c) * Np;
            for (int i = 0; i < Np; ++i) {
                double dr = 0, ds = 0;
                for (int j = 0; j < Np; ++j) {
                    dr += m->Dr[i * Np + j] * u[j];
                    ds += m->Ds[i * Np + j] * u[j];
                }
                long n = k * Np + i;
                double qx = sig * (m->rx[n] * dr + m->sx[n] * ds);
                double qy = sig * (m->ry[n] * dr + m->sy[n] * ds);
                for (int t = 0; t < Nf3; ++t) {
                    qx += m->LIFT[i * Nf3 + t] * jx[t][c];
                    qy += m->LIFT[i * Nf3 + t] * jy[t][c];
                }
                Q[((k * 2 + 0) * NF + c) * Np + i] = qx;
                Q[((k * 2 + 1) * NF + c) * Np + i] = qy;
            }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* right-hand side                                                        */
/* ---------------------------------------------------------------------- */

/* Normal viscous flux at a face node: visc_m = sigma- Q-.n (the element's
 * own trace) and the numerical flux visc_star = (sigma Q)*.n.
 * Interior: the central value 1/2 (sigma- Q- + sigma+ Q+).n.
 * Slip wall: the mean with the ghost gradient that the mirror ghost state
 * implies.  Mirroring a field across the wall flips the sign of its normal
 * derivative; rho and E are mirrored unchanged, so their (sigma Q)*.n is 0,
 * and the momentum m is mirrored to m - 2 (m.n) n, so of its normal
 * derivative g = (Q_x n_x + Q_y n_y) only the component along n survives:
 * (sigma Q)*.n = sigma- (g.n) n.
 * Far field: the element's own value sigma- Q-.n. */
static void viscous_face_flux(const oracle_mesh *m, long k, int f, int v, long kn, int vn,
                              double nx, double ny, double visc_m[NF], double visc_star[NF]) {
    const int Np = m->Np;
    const double *Q = m->Q, *eps = m->eps;
    double sig = sqrt(eps[k]);
    double g[NF];
    for (int c = 0; c < NF; ++c) {
        g[c] = nx * Q[((k * 2 + 0) * NF + c) * Np + v] + ny * Q[((k * 2 + 1) * NF + c) * Np + v];
        visc_m[c] = sig * g[c];
    }
    int code = m->bc[k * 3 + f];
    if (code == BC_INTERIOR) {
        double sigp = sqrt(eps[kn]);
        for (int c = 0; c < NF; ++c) {
            double gp = nx * Q[((kn * 2 + 0) * NF + c) * Np + vn] +
                        ny * Q[((kn * 2 + 1) * NF + c) * Np + vn];
            visc_star[c] = 0.5 * (visc_m[c] + sigp * gp);
        }
    } else if (code == BC_WALL) {
        double gn = g[1] * nx + g[2] * ny;
        visc_star[0] = 0.0;
        visc_star[1] = sig * gn * nx;
        visc_star[2] = sig * gn * ny;
        visc_star[3] = 0.0;
    } else {
        for (int c = 0; c < NF; ++c) visc_star[c] = visc_m[c];
    }
}

/* Right-hand side in the over-integrated weak form.  Per element k, with
 * phi_i the nodal basis and u = sum_j phi_j u_j:
 *   M_k dU/dt = V - S,
 *   V_i = int_k grad phi_i . (F(u), G(u)) dx
 *       = sum_q w_q J_q [dphi_i/dr (r_x F + r_y G) + dphi_i/ds (s_x F + s_y G)](x_q),
 *   S_i = oint_dk phi_i F*.n ds = sum_f sum_g w_g sJ_fg phi_i(x_fg) F*(u-, u+)_fg,
 *   M_k,ij = sum_q w_q J_q phi_i(x_q) phi_j(x_q),
 * with the metric terms, J, normals and sJ of the isoparametric map at each
 * cubature and face Gauss point, u- the element's face polynomial and u+
 * the neighbour's (or the boundary ghost state) at the same point; M_k is
 * solved by Cholesky factorisation.  Inviscid: the artificial viscosity is
 * defined for the nodal form only. */
static void cholesky_solve(int n, double *A, double *b) {
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
        d = sqrt(d);
        A[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = v / d;
        }
    }
    for (int i = 0; i < n; ++i) {       /* L y = b */
        double v = b[i];
        for (int k = 0; k < i; ++k) v -= A[i * n + k] * b[k];
        b[i] = v / A[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {  /* L^T x = y */
        double v = b[i];
        for (int k = i + 1; k < n; ++k) v -= A[k * n + i] * b[k];
        b[i] = v / A[i * n + i];
    }
}

void oracle_rhs_weak(const oracle_mesh *m, const double *U, double *rhs) {
    const oracle_weak *w = m->weak;
    const int Np = m->Np, Nfp = m->Nfp, nq = w->ncub, ng = w->ng;
    const double g = m->gamma;
#pragma omp parallel for
    for (long k = 0; k < m->K; ++k) {
        const double *xk = m->x + k * Np, *yk = m->y + k * Np;
        double V[NF][64] = {{0}}, S[NF][64] = {{0}}, M[64 * 64];
        for (int i = 0; i < Np * Np; ++i) M[i] = 0.0;
        for (int q = 0; q < nq; ++q) {
            const double *ph = w->Icub + q * Np, *pr = w->Drc + q * Np, *ps = w->Dsc + q * Np;
            double xr = 0, xs = 0, yr = 0, ys = 0, u[NF] = {0};
            for (int j = 0; j < Np; ++j) {
                xr += pr[j] * xk[j];
                xs += ps[j] * xk[j];
                yr += pr[j] * yk[j];
                ys += ps[j] * yk[j];
                for (int c = 0; c < NF; ++c) u[c] += ph[j] * U[(k * NF + c) * Np + j];
            }
            double J = xr * ys - xs * yr;
            double rx = ys / J, sx = -yr / J, ry = -xs / J, sy = xr / J;
            double F[NF], G[NF];
            euler_flux(g, u, F, G);
            double wJ = w->wq[q] * J;
            for (int c = 0; c < NF; ++c) {
                double a = wJ * (rx * F[c] + ry * G[c]);
                double b = wJ * (sx * F[c] + sy * G[c]);
                for (int i = 0; i < Np; ++i) V[c][i] += pr[i] * a + ps[i] * b;
            }
            for (int i = 0; i < Np; ++i)
                for (int j = 0; j < Np; ++j) M[i * Np + j] += wJ * ph[i] * ph[j];
        }
        for (int f = 0; f < 3; ++f) {
            int code = m->bc[k * 3 + f];
            long kn = m->EToE[k * 3 + f];
            int fn = m->EToF[k * 3 + f];
            for (int gq = 0; gq < ng; ++gq) {
                const double *lf = w->If + gq * Nfp;
                const double *pr = w->Drg + (f * ng + gq) * Np, *ps = w->Dsg + (f * ng + gq) * Np;
                double xr = 0, xs = 0, yr = 0, ys = 0;
                for (int j = 0; j < Np; ++j) {
                    xr += pr[j] * xk[j];
                    xs += ps[j] * xk[j];
                    yr += pr[j] * yk[j];
                    ys += ps[j] * yk[j];
                }
                double ax, ay;
                if (f == 0) { ax = yr; ay = -xr; }
                else if (f == 1) { ax = ys - yr; ay = xr - xs; }
                else { ax = -ys; ay = xs; }
                double sJ = sqrt(ax * ax + ay * ay), nx = ax / sJ, ny = ay / sJ;
                double um[NF] = {0}, up[NF] = {0}, fs[NF];
                for (int j = 0; j < Nfp; ++j) {
                    int v = m->Fmask[f * Nfp + j];
                    for (int c = 0; c < NF; ++c) um[c] += lf[j] * U[(k * NF + c) * Np + v];
                }
                if (code == BC_INTERIOR) {
                    /* the neighbour's face node Nfp-1-j sits on this face's node j */
                    for (int j = 0; j < Nfp; ++j) {
                        int v = m->Fmask[fn * Nfp + (Nfp - 1 - j)];
                        for (int c = 0; c < NF; ++c) up[c] += lf[j] * U[(kn * NF + c) * Np + v];
                    }
                } else {
                    oracle_ghost(g, code, um, nx, ny, m->freestream, up);
                }
                if (m->riemann == 1)
                    oracle_hllc_flux(g, um, up, nx, ny, fs);
                else
                    oracle_lf_flux(g, um, up, nx, ny, fs);
                double ws = w->wg[gq] * sJ;
                for (int j = 0; j < Nfp; ++j) {
                    int v = m->Fmask[f * Nfp + j];
                    for (int c = 0; c < NF; ++c) S[c][v] += ws * lf[j] * fs[c];
                }
            }
        }
        for (int c = 0; c < NF; ++c) {
            double A[64 * 64], b[64];
            for (int i = 0; i < Np * Np; ++i) A[i] = M[i];
            for (int i = 0; i < Np; ++i) b[i] = V[c][i] - S[c][i];
            cholesky_solve(Np, A, b);
            for (int i = 0; i < Np; ++i) rhs[(k * NF + c) * Np + i] = b[i];
        }
    }
}

/* dU/dt = -(r_x Dr F + s_x Ds F + r_y Dr G + s_y Ds G)
 *         + LIFT [Fscale (n.F(U-) - F*)]
 * where, with artificial viscosity, F and G include -sigma Q_x, -sigma Q_y
 * and F* includes -(sigma Q)*.n (viscous_face_flux). */
void oracle_rhs(oracle_mesh *m, const double *U, double *rhs) {
    if (m->weak) {
        oracle_rhs_weak(m, U, rhs);
        return;
    }
    const int Np = m->Np, Nfp = m->Nfp, Nf3 = 3 * m->Nfp;
    const double g = m->gamma;
    int av = m->av_enable || m->eps_override >= 0.0;
    if (av) {
        for (long k = 0; k < m->K; ++k) m->eps[k] = elem_eps(m, U, k);
        oracle_av_gradient(m, U, m->eps, m->Q);
    }
    const double *eps = m->eps, *Q = m->Q;
#pragma omp parallel for
    for (long k = 0; k < m->K; ++k) {
        double sig = av ? sqrt(eps[k]) : 0.0;
        double F[NF][64], G[NF][64];
        for (int i = 0; i < Np; ++i) {
            double u[NF], f[NF], gg[NF];
            for (int c = 0; c < NF; ++c) u[c] = U[(k * NF + c) * Np + i];
            if (m->no_euler_flux) {
                for (int c = 0; c < NF; ++c) f[c] = gg[c] = 0.0;
            } else {
                euler_flux(g, u, f, gg);
            }
            for (int c = 0; c < NF; ++c) {
                F[c][i] = f[c];
                G[c][i] = gg[c];
                if (av) {
                    F[c][i] -= sig * Q[((k * 2 + 0) * NF + c) * Np + i];
                    G[c][i] -= sig * Q[((k * 2 + 1) * NF + c) * Np + i];
                }
            }
        }
        /* surface flux differences, scaled by Fscale */
        double dfl[3 * 16][NF];
        for (int f = 0; f < 3; ++f)
            for (int j = 0; j < Nfp; ++j) {
                double um[NF], up[NF];
                long kn;
                int vn;
                face_states(m, U, k, f, j, um, up, &kn, &vn);
                long q = k * Nf3 + f * Nfp + j;
                double nx = m->nx[q], ny = m->ny[q];
                double fm[NF], fstar[NF], lam;
                if (m->no_euler_flux) {
                    for (int c = 0; c < NF; ++c) fm[c] = fstar[c] = 0.0;
                } else {
                    normal_flux(g, um, nx, ny, fm, &lam);
                    if (m->riemann == 1)
                        oracle_hllc_flux(g, um, up, nx, ny, fstar);
                    else
                        oracle_lf_flux(g, um, up, nx, ny, fstar);
                }
                int v = m->Fmask[f * Nfp + j];
                double visc_m[NF] = {0}, visc_star[NF] = {0};
                if (av) viscous_face_flux(m, k, f, v, kn, vn, nx, ny, visc_m, visc_star);
                for (int c = 0; c < NF; ++c) {
                    /* n.(F - sigma Q)(U-) - (F* - (sigma Q)*.n) */
                    double d = fm[c] - fstar[c];
                    if (av) d += -visc_m[c] + visc_star[c];
                    dfl[f * Nfp + j][c] = m->Fscale[q] * d;
                }
            }
        for (int c = 0; c < NF; ++c)
            for (int i = 0; i < Np; ++i) {
                double drf = 0, dsf = 0, drg = 0, dsg = 0;
                for (int j = 0; j < Np; ++j) {
                    drf += m->Dr[i * Np + j] * F[c][j];
                    dsf += m->Ds[i * Np + j] * F[c][j];
                    drg += m->Dr[i * Np + j] * G[c][j];
                    dsg += m->Ds[i * Np + j] * G[c][j];
                }
                long n = k * Np + i;
                double val = -(m->rx[n] * drf + m->sx[n] * dsf + m->ry[n] * drg + m->sy[n] * dsg);
                for (int t = 0; t < Nf3; ++t) val += m->LIFT[i * Nf3 + t] * dfl[t][c];
                rhs[(k * NF + c) * Np + i] = val;
            }
    }
}

/* ---------------------------------------------------------------------- */
/* time step, diagnostics, time integration                               */
/* ---------------------------------------------------------------------- */

/* dt = CFL / max over face nodes of
 *   1/2 (P+1)^2 Fscale (|v| + c) + 1/4 (P+1)^4 Fscale^2 eps_k.
 * *flag gets 1 if any node has a non-finite value, rho <= 0 or p <= 0. */
double oracle_dt(oracle_mesh *m, const double *U, int *flag) {
    const int Np = m->Np, Nf3 = 3 * m->Nfp;
    const double g = m->gamma;
    double P1 = m->P + 1.0;
    int av = m->av_enable || m->eps_override >= 0.0;
    double vmax = 0.0;
    int bad = 0;
    for (long k = 0; k < m->K; ++k) {
        for (int i = 0; i < Np; ++i) {
            double u[NF];
            for (int c = 0; c < NF; ++c) u[c] = U[(k * NF + c) * Np + i];
            double p = pressure(g, u);
            if (!(u[0] > 0.0) || !(p > 0.0) || !isfinite(u[1]) || !isfinite(u[2]) ||
                !isfinite(u[3]) || !isfinite(p))
                bad = 1;
        }
        double e = av ? elem_eps(m, U, k) : 0.0;
        for (int q = 0; q < Nf3; ++q) {
            int v = m->Fmask[q];
            double u[NF];
            for (int c = 0; c < NF; ++c) u[c] = U[(k * NF + c) * Np + v];
            double rho = u[0], ux = u[1] / rho, uy = u[2] / rho;
            double lam = sqrt(ux * ux + uy * uy) + sqrt(g * pressure(g, u) / rho);
            double fs = m->Fscale[k * Nf3 + q];
            double val = 0.5 * P1 * P1 * fs * lam + 0.25 * P1 * P1 * P1 * P1 * fs * fs * e;
            if (val > vmax) vmax = val;
        }
    }
    if (flag) *flag = bad;
    return m->cfl * (1.0 / vmax);
}

/* Conserved totals: sum_k sum_i w_ki U_ki with w_ki = sum_j M_ij J_kj. */
void oracle_totals(const oracle_mesh *m, const double *U, double out[NF]) {
    const int Np = m->Np;
    for (int c = 0; c < NF; ++c) out[c] = 0.0;
    for (long k = 0; k < m->K; ++k)
        for (int i = 0; i < Np; ++i) {
            double w = 0.0;
            for (int j = 0; j < Np; ++j) w += m->Mref[i * Np + j] * m->J[k * Np + j];
            for (int c = 0; c < NF; ++c) out[c] += w * U[(k * NF + c) * Np + i];
        }
}

/* Carpenter-Kennedy 2N-storage (5,4) coefficients. */
static const double RK_A[5] = {0.0,
                               -567301805773.0 / 1357537059087.0,
                               -2404267990393.0 / 2016746695238.0,
                               -3550918686646.0 / 2091501179385.0,
                               -1275806237668.0 / 842570457699.0};
static const double RK_B[5] = {1432997174477.0 / 9575080441755.0,
                               5161836677717.0 / 13612068292357.0,
                               1720146321549.0 / 2090206949498.0,
                               3134564353537.0 / 4481467310338.0,
                               2277821191437.0 / 14882151754819.0};

void oracle_rk_coefficients(double a[5], double b[5]) {
    for (int i = 0; i < 5; ++i) {
        a[i] = RK_A[i];
        b[i] = RK_B[i];
    }
}

/* nsteps LSERK steps.  dt_fixed > 0: that step; otherwise the CFL step from
 * U at the start of every step.  R and rhs are caller scratch of U's size.
 * Returns the simulated time; dt_minmax gets (min, max) of the steps used;
 * *flag the non-finite / non-positive state flag. */
double oracle_run(oracle_mesh *m, double *U, int nsteps, double dt_fixed,
                  double *R, double *rhs, double dt_minmax[2], int *flag) {
    const long n = (long)m->K * NF * m->Np;
    double t = 0.0;
    dt_minmax[0] = INFINITY;
    dt_minmax[1] = 0.0;
    *flag = 0;
    for (int step = 0; step < nsteps; ++step) {
        int bad = 0;
        double dt = dt_fixed > 0.0 ? dt_fixed : oracle_dt(m, U, &bad);
        if (dt_fixed > 0.0) (void)oracle_dt(m, U, &bad);
        *flag |= bad;
        if (dt < dt_minmax[0]) dt_minmax[0] = dt;
        if (dt > dt_minmax[1]) dt_minmax[1] = dt;
        for (int s = 0; s < 5; ++s) {
            oracle_rhs(m, U, rhs);
#pragma omp parallel for
            for (long i = 0; i < n; ++i) {
                R[i] = (s == 0) ? dt * rhs[i] : RK_A[s] * R[i] + dt * rhs[i];
                U[i] = U[i] + RK_B[s] * R[i];
            }
        }
        t += dt;
    }
    return t;
}

/* Residual infinity norm per field of rhs(U). */
void oracle_residual(oracle_mesh *m, const double *U, double *rhs, double out[NF]) {
    const int Np = m->Np;
    oracle_rhs(m, U, rhs);
    for (int c = 0; c < NF; ++c) out[c] = 0.0;
    for (long k = 0; k < m->K; ++k)
        for (int c = 0; c < NF; ++c)
            for (int i = 0; i < Np; ++i) {
                double a = fabs(rhs[(k * NF + c) * Np + i]);
                if (a > out[c]) out[c] = a;
            }
}

int oracle_abi_version(void) { return 1; }

#ifdef _OPENMP
#include <omp.h>
void oracle_set_threads(int n) { omp_set_num_threads(n); }
int oracle_max_threads(void) { return omp_get_max_threads(); }
#else
void oracle_set_threads(int n) { (void)n; }
int oracle_max_threads(void) { return 1; }
#endif
