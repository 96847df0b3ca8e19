"""Accuracy of the reduced-precision paths against the FP64 path.

Every solve here runs in the library's kernels; this module only reads the
resulting states back and evaluates diagnostics on the host:

* state error: relative L2 and maximum absolute difference against the FP64
  run of the same case at the same step;
* entropy error: the mass-weighted RMS of (s - s_inf) / s_inf with
  s = p / rho^gamma, which a smooth subsonic flow keeps at its
  discretisation error (the exact flow is isentropic);
* wall loads: lift and drag coefficients from the pressure integral over
  the wall faces (Gauss-Lobatto quadrature on the face nodes of the curved
  geometry), the minimum pressure coefficient and, on the upper surface,
  the shock position: the last upward crossing of the critical pressure
  coefficient C_p* (the flow behind it is subsonic to the trailing edge);
* freestream preservation on an all-curved mesh (a uniform state must stay
  uniform up to rounding) and the drift of the conserved totals on a
  periodic mesh.

The FP64 path these are measured against matches the FP64 oracle to 1e-12
(parity tests), so the differences are those of the reduced precision.
"""
from __future__ import annotations

import json
import math
import sys

import numpy as np

import meshgen

from . import dg

GAMMA = 1.4


def critical_cp(mach, gamma=GAMMA):
    """Pressure coefficient at which the isentropic local Mach number is 1."""
    g = gamma
    return 2.0 / (g * mach * mach) * (((2.0 + (g - 1.0) * mach * mach) / (g + 1.0)) ** (g / (g - 1.0)) - 1.0)


# -- host geometry -----------------------------------------------------------

def _legendre(n, t):
    """Legendre polynomials P_0..P_{n-1} at points t, shape (len(t), n)."""
    out = np.zeros((len(t), n))
    out[:, 0] = 1.0
    if n > 1:
        out[:, 1] = t
    for k in range(2, n):
        out[:, k] = ((2 * k - 1) * t * out[:, k - 1] - (k - 1) * out[:, k - 2]) / k
    return out


def _line_rule(t):
    """Quadrature weights and differentiation matrix of the Lagrange basis
    through the points t on [-1, 1]."""
    n = len(t)
    V = _legendre(n, t)
    m = np.zeros(n)
    m[0] = 2.0
    w = np.linalg.solve(V.T, m)
    # derivative of the Legendre basis: P_k' from the recurrence
    # (2k+1) P_k = P_{k+1}' - P_{k-1}'
    dV = np.zeros_like(V)
    for k in range(1, n):
        dV[:, k] = (2 * k - 1) * V[:, k - 1] + (dV[:, k - 2] if k >= 2 else 0.0)
    D = dV @ np.linalg.inv(V)
    return w, D


class Geometry:
    """Mass weights and wall-face quadrature of a case, in the library's
    node order."""

    def __init__(self, case):
        P = case.P
        ops = dg.reference_operators(P)
        r, s = dg.reference_nodes(P)
        fm = dg.face_nodes(P)
        x, y = case.x, case.y
        Dr, Ds, Vinv = ops["Dr"], ops["Ds"], ops["Vinv"]
        xr, xs, yr, ys = x @ Dr.T, x @ Ds.T, y @ Dr.T, y @ Ds.T
        J = xr * ys - xs * yr
        M = Vinv.T @ Vinv
        self.wmass = J @ M.T                      # w_ki = sum_j M_ij J_kj
        self.area = float(self.wmass.sum())
        # wall faces: (element, face) pairs and their node quadrature
        bc = case.mesh.bc
        ks, fs = np.nonzero(bc == meshgen.BC_WALL)
        self.wall_k, self.wall_f = ks, fs
        nodes, wts, nx, ny, xw, yw = [], [], [], [], [], []
        for f in range(3):
            sel = fs == f
            if not sel.any():
                continue
            ids = fm[f]
            # edge parameter in the face's counter-clockwise direction
            t = (r, s, -s)[f][ids]
            w1, D1 = _line_rule(t)
            xe, ye = x[ks[sel]][:, ids], y[ks[sel]][:, ids]
            dx, dy = xe @ D1.T, ye @ D1.T
            L = np.hypot(dx, dy)
            nodes.append((ks[sel], ids))
            wts.append(L * w1)
            nx.append(dy / L)        # outward for a counter-clockwise element
            ny.append(-dx / L)
            xw.append(xe)
            yw.append(ye)
        self._wall = list(zip(nodes, wts, nx, ny, xw, yw))

    def wall_loads(self, U, freestream, gamma=GAMMA):
        """Pressure force on the walls as lift/drag coefficients (reference
        length 1), the minimum pressure coefficient and the upper-surface
        shock position (last upward crossing of C_p*, NaN without one);
        None without walls."""
        if not self._wall:
            return None
        q = np.asarray(freestream, dtype=np.float64)
        rho0, u0, v0 = q[0], q[1] / q[0], q[2] / q[0]
        V2 = u0 * u0 + v0 * v0
        p0 = (gamma - 1.0) * (q[3] - 0.5 * rho0 * V2)
        qdyn = 0.5 * rho0 * V2
        mach = math.sqrt(V2 / (gamma * p0 / rho0))
        Fx = Fy = 0.0
        xs_all, ys_all, cps = [], [], []
        for (ke, ids), w, nx, ny, xe, ye in self._wall:
            Uf = U[ke][:, :, ids]                  # (n, 4, Nfp)
            rho, mx, my, E = Uf[:, 0], Uf[:, 1], Uf[:, 2], Uf[:, 3]
            p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / rho)
            # force on the body: pressure along the element's outward normal
            Fx += float((p * nx * w).sum())
            Fy += float((p * ny * w).sum())
            xs_all.append(xe.ravel())
            ys_all.append(ye.ravel())
            cps.append(((p - p0) / qdyn).ravel())
        ca, sa = u0 / math.sqrt(V2), v0 / math.sqrt(V2)
        CD = (Fx * ca + Fy * sa) / qdyn
        CL = (-Fx * sa + Fy * ca) / qdyn
        xw, yw, cp = np.concatenate(xs_all), np.concatenate(ys_all), np.concatenate(cps)
        out = dict(CL=CL, CD=CD, cp_min=float(cp.min()), shock_x=float("nan"))
        up = yw > 0
        if up.sum() > 1:
            order = np.argsort(xw[up], kind="stable")
            xu, cu = xw[up][order], cp[up][order]
            keep = np.concatenate([[True], np.diff(xu) > 1e-12])
            xu, cu = xu[keep], cu[keep]
            cstar = critical_cp(mach, gamma)
            ups = np.nonzero((cu[:-1] < cstar) & (cu[1:] >= cstar))[0]
            if ups.size:
                i = int(ups[-1])
                out["shock_x"] = float(xu[i] + (cstar - cu[i]) / (cu[i + 1] - cu[i]) * (xu[i + 1] - xu[i]))
        return out

    def entropy_error(self, U, freestream, gamma=GAMMA):
        q = np.asarray(freestream, dtype=np.float64)
        p0 = (gamma - 1.0) * (q[3] - 0.5 * (q[1] ** 2 + q[2] ** 2) / q[0])
        s0 = p0 / q[0] ** gamma
        rho = U[:, 0]
        p = (gamma - 1.0) * (U[:, 3] - 0.5 * (U[:, 1] ** 2 + U[:, 2] ** 2) / rho)
        e = (p / rho ** gamma - s0) / s0
        return float(math.sqrt(max((self.wmass * e * e).sum(), 0.0) / self.area))

    def totals(self, U):
        return np.einsum("ki,kci->c", self.wmass, U)


def state_errors(U, Uref):
    d = U - Uref
    return dict(rel_l2=float(np.linalg.norm(d.ravel()) / np.linalg.norm(Uref.ravel())),
                max_abs=float(np.abs(d).max()))


# -- runs ------------------------------------------------------------------

def run_stations(case, precision, stations, device="cuda:0"):
    """Run the case from its start, returning the host state (FP64 copy) and
    simulated time at each step count in ``stations``."""
    import torch
    sol = dg.Solver.from_case(case, precision, device=device)
    U = sol.state(case.U0)
    out, done = [], 0
    for n in stations:
        st = sol.run(U, n - done, check=False)
        torch.cuda.synchronize()
        done = n
        out.append(dict(step=n, status=st.status, t=st.t if not out else out[-1]["t"] + st.t,
                        U=U.double().cpu().numpy()))
        if case.av and st.status == 0:
            out[-1]["viscous_elements"] = int((sol.viscosity(U) > 0).sum().item())
        print(f"[{case.name} {precision}] step {n} t {out[-1]['t']:.5f} status {st.status}",
              file=sys.stderr, flush=True)
        if st.status != 0:
            break
    sol.close()
    return out


def precision_report(case, stations, precisions=("fp32", "bf16x3"), loads=True):
    """FP64 run and each reduced-precision run of ``case``, compared at every
    station: state errors, entropy errors, wall loads."""
    geo = Geometry(case)
    ref = run_stations(case, "fp64", stations)
    runs = {p: run_stations(case, p, stations) for p in precisions}
    rows = []
    for i, r64 in enumerate(ref):
        row = dict(step=r64["step"], t=r64["t"], fp64=dict(
            status=r64["status"], entropy_error=geo.entropy_error(r64["U"], case.freestream)))
        if "viscous_elements" in r64:
            row["fp64"]["viscous_elements"] = r64["viscous_elements"]
        if loads:
            row["fp64"]["wall"] = geo.wall_loads(r64["U"], case.freestream)
        for p, rr in runs.items():
            if i >= len(rr):
                row[p] = dict(status="stopped earlier")
                continue
            e = dict(status=rr[i]["status"], t=rr[i]["t"], **state_errors(rr[i]["U"], r64["U"]),
                     entropy_error=geo.entropy_error(rr[i]["U"], case.freestream))
            if "viscous_elements" in rr[i]:
                e["viscous_elements"] = rr[i]["viscous_elements"]
            if loads:
                e["wall"] = geo.wall_loads(rr[i]["U"], case.freestream)
            row[p] = e
        rows.append(row)
    return dict(case=case.name, K=case.K, P=case.P, stations=list(stations), rows=rows)


def freestream_and_conservation(scale=1.0, steps=200, precisions=("fp64", "fp32", "bf16x3")):
    """Freestream preservation on the all-curved periodic mesh and the drift
    of the conserved totals on the straight periodic vortex mesh."""
    out = {}
    r, s = dg.reference_nodes(5)
    curved = meshgen.make_case("roofline_curved", r, s, scale=scale)
    q = np.asarray(curved.freestream, dtype=np.float64)
    curved.U0 = meshgen.uniform((curved.K, curved.Np), q)
    vortex = meshgen.make_case("roofline", r, s, scale=scale)
    geo = Geometry(vortex)
    T0 = geo.totals(vortex.U0)
    for p in precisions:
        f = run_stations(curved, p, [steps])[-1]
        dev = np.abs(f["U"] - q[None, :, None]).max(axis=(0, 2)) / np.maximum(np.abs(q), 1.0)
        v = run_stations(vortex, p, [steps])[-1]
        T = geo.totals(v["U"])
        out[p] = dict(freestream_max_rel_dev=[float(x) for x in dev], freestream_status=f["status"],
                      totals_rel_drift=[float(x) for x in np.abs(T - T0) / np.maximum(np.abs(T0), 1e-300)],
                      vortex_status=v["status"], t=v["t"])
    return dict(K_curved=curved.K, K_vortex=vortex.K, P=5, steps=steps, results=out)


def _jsonable(x):
    if isinstance(x, dict):
        return {k: _jsonable(v) for k, v in x.items() if k != "U"}
    if isinstance(x, list):
        return [_jsonable(v) for v in x]
    if isinstance(x, (np.floating, np.integer)):
        return x.item()
    return x


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="accuracy of the reduced-precision paths vs FP64")
    ap.add_argument("report", choices=["cylinder", "airfoil", "roofline"])
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--stations", type=int, default=4)
    ap.add_argument("--start", default=None, choices=["freestream", "potential", "damped"],
                    help="initial state of the cylinder/airfoil (default: the case's own)")
    ap.add_argument("--kappa", type=float, default=None, help="sensor half-width (default: the case's own)")
    ap.add_argument("--precisions", default="fp32,bf16x3", help="reduced precisions compared with FP64")
    a = ap.parse_args(argv)
    if a.report == "roofline":
        res = freestream_and_conservation(a.scale, a.steps or 200)
    else:
        P = {"cylinder": 4, "airfoil": 3}[a.report]
        r, s = dg.reference_nodes(P)
        case = meshgen.make_case(a.report, r, s, scale=a.scale,
                                 **({"start": a.start} if a.start else {}))
        if a.kappa is not None:
            case.av_kappa = a.kappa
        n = a.steps or case.steps
        stations = sorted({max(1, round(n * (i + 1) / a.stations)) for i in range(a.stations)})
        res = precision_report(case, stations, precisions=tuple(a.precisions.split(",")))
        res["av_kappa"] = case.av_kappa
    print(json.dumps(_jsonable(res)), flush=True)


if __name__ == "__main__":
    main()
