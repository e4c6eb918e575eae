"""The assembled effective field, energies and RK4 LLG (paper Eqs. heff, hms_d, llg).

H_eff = H_ex + H_ms (+ a uniform applied field), Eq. heff; anisotropy is not
part of any workload here. Two levels of the potential:

* ``method="direct"`` -- the definition, Eqs. hms_d2/hms_d2b: the point-charge
  superposition with the periodic Green's function over all node pairs,
      u_n = (1/4 pi)[ sum_{k != n} G^p(r_n - r_k) q_k + G_reg(0) q_n ] + u_Z,n,
  (reading: the k = n term of Eq. hms_d2 keeps only the self images).
* ``method="aim"`` -- the paper's four-step AIM (oracle.aim) plus u_Z.

u_Z is the element-exact correction of Eq. hms_d2b. The charges of the
body are split by element: each tetrahedron e carries its constant volume
density rho_e = -Ms_e div(m)_e and, on those of its faces that are surface
faces of the body (not glued to another tetrahedron of the same material
after LCA merging: outer boundary and material interfaces, Sec. 3.2.1),
the linear surface density sigma = Ms_e m.n. Their nodal shares q_i^(e)
(weights lambda_i, consistent face mass) add up to the weak-form charges.
For every tetrahedron whose centroid lies within kappa * (mean edge length)
of r_n in the minimum image (the paper's radius "based on the average edge
length", Sec. 3.2.2), the exact potential of e replaces the point charges
that e contributes to the other nodes:
      u_Z,n = (1/4 pi) sum_e [ int_e rho_e / R + sum_{f surface} int_f sigma / R
                               - sum_{i in e, i != n} q_i^(e) / |r_n - r_i*| ].
It acts on m directly (three sparse blocks), separate from the precorrection.

LLG (Eq. llg, reading of the garbled "M x M_n x H"): unit-vector
Landau-Lifshitz form dm/dt = -gamma0/(1+alpha^2) [m x H + alpha m x (m x H)],
gamma0 = mu0 * 1.76086e11 m/(A s) (the paper gives no value), classic RK4
with the norm restored after each full step. The paper itself integrates
implicitly (midpoint or BDF with Newton and a preconditioned Krylov solver,
Sec. 2.2); ``implicit_midpoint`` is that rule written out plainly: each step
solves x = m + dt f((m + x)/2) by Newton's method with the exact Jacobian
(the field is linear in m, so H = A m + H_app with A assembled densely on
small meshes) and a dense linear solve; the rule keeps |m| by itself.
``implicit_midpoint_adaptive`` and ``implicit_bdf2_adaptive`` add the
paper's time-step control (Sec. 2.2, Sec. 5) as predictor-corrector pairs.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from . import periodic, fem, pgf as pgfmod, aim as aimmod, elem

MU0 = fem.MU0
GAMMA0 = MU0 * 1.76086e11


def mean_edge_length(xyz, tets):
    e = np.concatenate([tets[:, [i, j]] for i in range(4) for j in range(i + 1, 4)])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return float(np.mean(np.linalg.norm(xyz[e[:, 0]] - xyz[e[:, 1]], axis=1)))


class Oracle:
    def __init__(self, prob, order_p=None, near_boxes=None, z0_radius=None, tol_rel=1e-9,
                 eta=None, with_aim=True):
        self.prob = prob
        self.mask = int(prob.periodic)
        self.L = np.asarray(prob.L, dtype=np.float64)
        self.p = prob.order_p if order_p is None else order_p
        self.r_b = prob.near_boxes if near_boxes is None else near_boxes
        self.kappa = prob.z0_radius if z0_radius is None else z0_radius
        self.eta = eta
        xyz, tets = prob.xyz, prob.tets.astype(np.int64)
        self.uk, self.reps, self.n_pbc = periodic.unknowns(xyz, self.mask, self.L, tol_rel)
        self.n = self.reps.size
        self.ops = fem.LocalOperators(xyz, tets, prob.region, prob.Ms, prob.Aex, self.uk, self.n)
        self.pos = periodic.remap(xyz[self.reps], self.mask, self.L)
        self.hbar = mean_edge_length(xyz, tets)
        self.aim = (aimmod.AIM(self.pos, self.mask, self.L, prob.grid, self.p, self.r_b, eta)
                    if with_aim else None)
        self._greg0 = pgfmod.greg0(self.mask, self.L, eta) if self.mask else 0.0
        self._cache = {}

    # -- inputs ----------------------------------------------------------
    def unknown_values(self, m_nodes):
        return np.asarray(m_nodes, dtype=np.float64)[self.reps]

    # -- element-exact correction ------------------------------------------
    def _minimg(self, d):
        d = np.array(d, copy=True)
        for a in range(3):
            if (self.mask >> a) & 1:
                d[..., a] -= self.L[a] * np.round(d[..., a] / self.L[a])
        return d

    def _surface_faces(self):
        """[T,4] bool: face opposite local vertex a is a surface face of the body."""
        tets = self.prob.tets.astype(np.int64)
        U = self.uk[tets]
        keys, owner, opp = [], [], []
        for a in range(4):
            tri = np.sort(np.delete(U, a, axis=1), axis=1)
            keys.append(tri)
            owner.append(np.arange(tets.shape[0]))
            opp.append(np.full(tets.shape[0], a))
        keys = np.concatenate(keys)
        owner = np.concatenate(owner)
        opp = np.concatenate(opp)
        _, inv, cnt = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
        inv = inv.ravel()
        if cnt.max() > 2:
            raise ValueError("a face is shared by more than two tetrahedra")
        reg = np.asarray(self.prob.region)[owner]
        # two sides of one face: interior unless the regions differ
        first = np.full(cnt.size, -1, dtype=np.int64)
        other = np.full(cnt.size, -1, dtype=np.int64)
        for i in range(keys.shape[0]):
            if first[inv[i]] < 0:
                first[inv[i]] = i
            else:
                other[inv[i]] = i
        surf = np.ones(keys.shape[0], dtype=bool)
        both = other >= 0
        same = np.zeros(cnt.size, dtype=bool)
        same[both] = reg[first[both]] == reg[other[both]]
        surf[same[inv]] = False
        out = np.zeros((tets.shape[0], 4), dtype=bool)
        out[owner, opp] = surf
        return out

    def z0(self, rows):
        """Three sparse blocks [len(rows), N'] with u_Z[rows] = sum_c Z[c] @ m[:, c]."""
        key = ("z0", tuple(np.asarray(rows).tolist()))
        if key in self._cache:
            return self._cache[key]
        if "surf" not in self._cache:
            self._cache["surf"] = self._surface_faces()
        surf_all = self._cache["surf"]
        prob = self.prob
        xyz, tets = prob.xyz, prob.tets.astype(np.int64)
        X = xyz[tets]
        cen = X.mean(axis=1)
        rad = self.kappa * self.hbar
        rows = np.asarray(rows)
        robs = xyz[self.reps[rows]]
        # periodic KD-tree: wrap periodic axes into [0, L), pad the others
        lo = np.minimum(cen.min(axis=0), robs.min(axis=0))
        ext = np.maximum(cen.max(axis=0), robs.max(axis=0)) - lo
        box = np.where([(self.mask >> a) & 1 for a in range(3)], self.L, 4 * ext + 4 * rad)
        tree = cKDTree(np.mod(cen - lo, box), boxsize=box)
        lists = tree.query_ball_point(np.mod(robs - lo, box), r=rad)
        pr = np.concatenate([np.full(len(l), i) for i, l in enumerate(lists)]).astype(np.int64)
        pe = np.concatenate([np.asarray(l, dtype=np.int64) for l in lists])
        n_obs = rows[pr]
        r = robs[pr]
        shift = self._minimg(cen[pe] - r) - (cen[pe] - r)
        Xs = X[pe] + shift[:, None, :]
        U = self.uk[tets[pe]]                                     # [P,4]
        at = (U == n_obs[:, None])
        vertex = np.where(at.any(axis=1), np.argmax(at, axis=1), -1)
        if np.any(vertex >= 0):
            hit = Xs[np.arange(pe.size), np.maximum(vertex, 0)]
            bad = (vertex >= 0) & (np.linalg.norm(hit - r, axis=1) > 1e-6 * self.hbar)
            if np.any(bad):
                raise ValueError("element vertex maps to the observer at another image")
        grad = self.ops.grad[pe]                                  # [P,4,3]
        ms = np.asarray(prob.Ms, dtype=np.float64)[prob.region[pe]]
        V = self.ops.V[pe]
        dist = np.linalg.norm(r[:, None, :] - Xs, axis=2)          # [P,4]
        g0 = np.where(at, 0.0, 1.0 / np.maximum(dist, 1e-300))     # point kernel, i != n
        # volume charge: coefficient of m_j is -Ms grad(lambda_j)
        IV = elem.tet_inv_r(r, Xs, vertex)
        exact = -(ms * IV)[:, None, None] * grad                     # [P,4(j),3]
        point = -(ms * V / 4.0 * g0.sum(axis=1))[:, None, None] * grad
        surf = surf_all[pe]
        for a in range(4):
            sel = np.nonzero(surf[:, a])[0]
            if sel.size == 0:
                continue
            loc = np.array([b for b in range(4) if b != a])
            T = Xs[sel][:, loc, :]
            nrm = np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0])
            area = 0.5 * np.linalg.norm(nrm, axis=1)
            nhat = nrm / (2 * area)[:, None]
            outward = np.einsum("pi,pi->p", nhat, T[:, 0] - Xs[sel][:, a, :]) > 0
            nhat[~outward] *= -1
            vloc = np.where(vertex[sel, None] == loc[None, :])
            tv = np.full(sel.size, -1)
            tv[vloc[0]] = vloc[1]
            If = elem.tri_lambda_inv_r(r[sel], T, tv)              # [p,3(l)]
            for li, j in enumerate(loc):
                exact[sel, j, :] += (ms[sel] * If[:, li])[:, None] * nhat
                # share of node i in the face charge of m_j: (A/12)(1 + delta_ij)
                share = sum(g0[sel, i] * (1.0 + (i == j)) for i in loc)
                point[sel, j, :] += (ms[sel] * area / 12.0 * share)[:, None] * nhat
        coef = (exact - point) / (4 * np.pi)
        rr = np.repeat(pr, 4)
        cc = U.ravel()
        out = [sp.csr_matrix((coef[:, :, c].ravel(), (rr, cc)), shape=(rows.size, self.n))
               for c in range(3)]
        self._cache[key] = out
        return out

    # -- potentials ----------------------------------------------------------
    def potential(self, m, rows=None, method="aim", z0=True):
        """Corrected potential u [A] at rows (sorted unknown ids) or everywhere."""
        rows = np.arange(self.n) if rows is None else np.asarray(rows)
        q = self.ops.charges(m)
        if method == "aim":
            key = ("P", tuple(rows.tolist()))
            if key not in self._cache:
                self._cache[key] = self.aim.precorrection(rows)
            U = self.aim.convolve(self.aim.project(q))
            u = (self.aim.interpolate(U, rows) + self._cache[key] @ q) / (4 * np.pi)
        elif method == "direct":
            u = self._direct(q, rows)
        else:
            raise ValueError(method)
        if z0:
            Z = self.z0(rows)
            u = u + sum(Z[c] @ m[:, c] for c in range(3))
        return u

    def _direct(self, q, rows):
        out = np.empty(rows.size)
        pos = self.pos
        for i0 in range(0, rows.size, 64):
            rr = rows[i0:i0 + 64]
            d = (pos[rr][:, None, :] - pos[None, :, :]).reshape(-1, 3)
            same = (rr[:, None] == np.arange(self.n)[None, :]).ravel()
            g = np.empty(d.shape[0])
            g[same] = self._greg0
            g[~same] = pgfmod.pgf(d[~same], self.mask, self.L, self.eta)
            out[i0:i0 + 64] = g.reshape(rr.size, self.n) @ q
        return out / (4 * np.pi)

    # -- fields ------------------------------------------------------------
    def heff(self, m, rows=None, method="aim", terms=("ex", "ms"), h_app=None, z0=True):
        """H_eff [len(rows),3] (A/m) for unit vectors m [N',3] on the unknowns."""
        m = np.asarray(m, dtype=np.float64)
        rows_ = np.arange(self.n) if rows is None else np.asarray(rows)
        H = np.zeros((rows_.size, 3))
        if "ex" in terms:
            H += self.ops.exchange(m)[rows_]
        if "ms" in terms:
            ring = np.arange(self.n) if rows is None else self.ops.neighbours(rows_)
            u = np.zeros(self.n)
            u[ring] = self.potential(m, ring, method, z0)
            H += self.ops.gradient_field(u, rows_)
        if h_app is not None:
            H += np.asarray(h_app, dtype=np.float64)[None, :]
        return H

    def charges(self, m):
        return self.ops.charges(np.asarray(m, dtype=np.float64))

    def energy(self, m, method="aim", h_app=None):
        """(E_ex, E_ms, E_zeeman) in J."""
        e_ex = self.ops.exchange_energy(m)
        q = self.ops.charges(m)
        u = self.potential(m, None, method)
        e_ms = 0.5 * MU0 * float(q @ u)
        e_z = 0.0
        if h_app is not None:
            e_z = -MU0 * float(np.sum(self.ops.mu[:, None] * m * np.asarray(h_app)[None, :]))
        return e_ex, e_ms, e_z

    # -- LLG -------------------------------------------------------------
    def llg_rhs(self, m, H, alpha):
        mxh = np.cross(m, H)
        return -GAMMA0 / (1 + alpha * alpha) * (mxh + alpha * np.cross(m, mxh))

    def rk4(self, m, dt, alpha, n_steps, method="aim", terms=("ex", "ms"), h_app=None):
        m = np.array(m, dtype=np.float64, copy=True)

        def f(mm):
            return self.llg_rhs(mm, self.heff(mm, None, method, terms, h_app), alpha)
        for _ in range(n_steps):
            k1 = f(m)
            k2 = f(m + 0.5 * dt * k1)
            k3 = f(m + 0.5 * dt * k2)
            k4 = f(m + dt * k3)
            m = m + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
            m /= np.linalg.norm(m, axis=1, keepdims=True)
        return m

    # -- implicit midpoint (small meshes: dense operators) ------------------
    def field_matrix(self, method="aim", terms=("ex", "ms")):
        """Dense A [3N', 3N'] with H(m) = A m (row-major [node][component]):
        the field without the applied part is linear in m (Eqs. hex, hms_d)."""
        n3 = 3 * self.n
        A = np.empty((n3, n3))
        for j in range(n3):
            e = np.zeros(n3)
            e[j] = 1.0
            A[:, j] = self.heff(e.reshape(self.n, 3), None, method, terms).ravel()
        return A

    @staticmethod
    def _cross_matrix(v):
        """[N,3,3] matrices C with C[n] w = v[n] x w."""
        C = np.zeros(v.shape[:1] + (3, 3))
        C[:, 0, 1], C[:, 0, 2] = -v[:, 2], v[:, 1]
        C[:, 1, 0], C[:, 1, 2] = v[:, 2], -v[:, 0]
        C[:, 2, 0], C[:, 2, 1] = -v[:, 1], v[:, 0]
        return C

    def implicit_midpoint(self, m, dt, alpha, n_steps, method="aim", terms=("ex", "ms"),
                          h_app=None, tol=1e-14, max_newton=30, A=None):
        """n_steps of x = m + dt f((m + x)/2), f the right side of Eq. llg;
        Newton on G(x) = x - m - dt f(mb), mb = (m + x)/2, with
        dG/dx = I - (dt/2) df/dmb,
        df/dmb w = c [w x H + mb x (A w) + alpha (w x (mb x H) + mb x (w x H)
                   + mb x (mb x (A w)))],  c = -gamma0/(1 + alpha^2).
        Returns the final m and the Newton iterations of each step."""
        n = self.n
        A = self.field_matrix(method, terms) if A is None else A
        b = np.zeros(3) if h_app is None else np.asarray(h_app, dtype=np.float64)
        c = -GAMMA0 / (1 + alpha * alpha)
        m = np.array(m, dtype=np.float64, copy=True)
        iters = []
        for _ in range(n_steps):
            x = m.copy()
            for it in range(max_newton):
                mb = 0.5 * (m + x)
                H = (A @ mb.ravel()).reshape(n, 3) + b[None, :]
                mxh = np.cross(mb, H)
                G = x - m - dt * c * (mxh + alpha * np.cross(mb, mxh))
                if np.abs(G).max() <= tol:
                    break
                CH, CM, CMH = self._cross_matrix(H), self._cross_matrix(mb), self._cross_matrix(mxh)
                local = -CH - alpha * CMH - alpha * CM @ CH       # [N,3,3], acts on w
                left = CM + alpha * CM @ CM                       # [N,3,3], acts on A w
                J = np.zeros((3 * n, 3 * n))
                for k in range(n):
                    J[3 * k:3 * k + 3, 3 * k:3 * k + 3] += local[k]
                    J[3 * k:3 * k + 3, :] += left[k] @ A[3 * k:3 * k + 3, :]
                dG = np.eye(3 * n) - 0.5 * dt * c * J
                x = x - np.linalg.solve(dG, G.ravel()).reshape(n, 3)
            else:
                raise RuntimeError("implicit midpoint: Newton did not converge")
            iters.append(it)
            m = x
        return m, iters

    # -- step-size-adaptive implicit midpoint -------------------------------
    LTE_C = 1.0 / 12.0   # midpoint rule: x - y(t+h) = C h^3 y''' for a linear right side

    @staticmethod
    def predictor_constant(h, h1, h2):
        """C_p with x_p - y(t+h) = C_p h^3 y''' for the predictor
        x_p = m + h ((1 + r) s1 - r s2), r = (h + h1) / (h1 + h2), where
        s1 = (m - m_prev) / h1 and s2 are the midpoint slopes of the last two
        steps (h1 the latest) and y the exact solution through the current m.
        The past states are the rule's own output, each off y by the local
        errors of the steps since (C h_i^3 y''' apiece), so a slope s_i equals
        y' at its step's midpoint plus (1/24 + C) h_i^2 y''' (1/24 from the
        chord, C from its own step's error); the line through the two midpoint
        values misses y' at the new midpoint by -y''' a b / 2, a and b the
        distances from the new midpoint to the two old ones; the midpoint
        quadrature of the new step adds -h^3 y''' / 24."""
        a = 0.5 * (h + h1)
        b = a + 0.5 * (h1 + h2)
        r = (h + h1) / (h1 + h2)
        k = 1.0 / 24.0 + Oracle.LTE_C
        return (-0.5 * a * b + k * ((1.0 + r) * h1 * h1 - r * h2 * h2)) / (h * h) - 1.0 / 24.0

    def implicit_midpoint_adaptive(self, m, t_end, dt0, alpha, lte_tol, method="aim",
                                   terms=("ex", "ms"), h_app=None, tol=1e-13, max_newton=10,
                                   A=None, max_steps=100000):
        """The midpoint rule of ``implicit_midpoint`` with an adaptive step, as a
        predictor-corrector pair (the time-step adaptive midpoint scheme of
        Sec. 2.2 and Sec. 5; the paper gives no formulas, the ones here are
        this oracle's reading):

        * predictor x_p: the midpoint slopes of the last two accepted steps
          extrapolated linearly to the new step's midpoint (one slope: that
          slope; none: x_p = m);
        * corrector x_c: the midpoint rule solved by Newton from x_p, converged
          when the rms of the residual is <= tol; no convergence within
          max_newton iterations (or a residual three times its first value)
          halves the step and retries;
        * from the third accepted step on, the local error estimate
          E = |C / (C - C_p)| rms(x_c - x_p) (Milne's device, C = 1/12, C_p from
          ``predictor_constant``); E > lte_tol rejects the step;
        * next step: h * min(2, max(0.2, 0.9 (lte_tol / E)^(1/3))), at most
          0.9 h after a rejection; without an estimate the step is kept; the
          last step is shortened to end at t_end;
        * an accepted state is renormalised per node (the rule keeps |m| up to
          the Newton residual) before it enters the slope history.

        Returns (m, info) with info["dts"] the accepted steps, info["lte"] their
        estimates (None for the first two), info["newton"] the Newton
        iterations of each accepted step, info["rejected"], info["dt_next"]."""
        n = self.n
        A = self.field_matrix(method, terms) if A is None else A
        b = np.zeros(3) if h_app is None else np.asarray(h_app, dtype=np.float64)
        c = -GAMMA0 / (1 + alpha * alpha)
        m = np.array(m, dtype=np.float64, copy=True)
        rms = np.sqrt(3.0 * n)

        def residual(x):
            mb = 0.5 * (m + x)
            H = (A @ mb.ravel()).reshape(n, 3) + b[None, :]
            mxh = np.cross(mb, H)
            return x - m - dt_try * c * (mxh + alpha * np.cross(mb, mxh)), mb, H, mxh

        def newton(x):
            g0 = None
            for it in range(max_newton + 1):
                G, mb, H, mxh = residual(x)
                g = np.linalg.norm(G) / rms
                if g <= tol:
                    return x, it
                if it == max_newton or not np.isfinite(g) or (g0 is not None and g > 3 * g0):
                    return None, it
                g0 = g if g0 is None else g0
                CH, CM, CMH = self._cross_matrix(H), self._cross_matrix(mb), self._cross_matrix(mxh)
                local = -CH - alpha * CMH - alpha * CM @ CH
                left = CM + alpha * CM @ CM
                J = np.zeros((3 * n, 3 * n))
                for k in range(n):
                    J[3 * k:3 * k + 3, 3 * k:3 * k + 3] += local[k]
                    J[3 * k:3 * k + 3, :] += left[k] @ A[3 * k:3 * k + 3, :]
                dG = np.eye(3 * n) - 0.5 * dt_try * c * J
                x = x - np.linalg.solve(dG, G.ravel()).reshape(n, 3)
            return None, max_newton

        t, dt = 0.0, float(dt0)
        slopes = []                                  # [(s, h)], latest first
        info = dict(dts=[], lte=[], newton=[], rejected=0, dt_next=dt)
        while t_end - t > 1e-12 * t_end:
            if len(info["dts"]) >= max_steps:
                raise RuntimeError("adaptive midpoint: step limit")
            dt_try = min(dt, t_end - t)
            if dt_try < 1e-9 * t_end:
                raise RuntimeError("adaptive midpoint: time step underflow")
            if len(slopes) >= 2:
                (s1, h1), (s2, h2) = slopes[0], slopes[1]
                r = (dt_try + h1) / (h1 + h2)
                xp = m + dt_try * ((1 + r) * s1 - r * s2)
            elif slopes:
                xp = m + dt_try * slopes[0][0]
            else:
                xp = m.copy()
            x, its = newton(xp.copy())
            if x is None:
                info["rejected"] += 1
                dt = 0.5 * dt_try
                continue
            est = None
            if len(slopes) >= 2:
                cp = self.predictor_constant(dt_try, slopes[0][1], slopes[1][1])
                est = abs(self.LTE_C / (self.LTE_C - cp)) * np.linalg.norm(x - xp) / rms
                fac = 0.9 * (lte_tol / est) ** (1.0 / 3.0) if est > 0 else 2.0
                if est > lte_tol:
                    info["rejected"] += 1
                    dt = dt_try * max(0.2, min(0.9, fac))
                    continue
                dt_new = dt_try * min(2.0, max(0.2, fac))
            else:
                dt_new = dt
            x = x / np.linalg.norm(x, axis=1, keepdims=True)
            slopes.insert(0, ((x - m) / dt_try, dt_try))
            del slopes[2:]
            m = x
            t += dt_try
            info["dts"].append(dt_try)
            info["lte"].append(est)
            info["newton"].append(its)
            dt = dt_new
        info["dt_next"] = dt
        return m, info

    # -- step-size-adaptive BDF2 -------------------------------------------
    @staticmethod
    def bdf2_coefficients(h, h1):
        """Variable-step BDF2 from y_n (step h1 before it: y_{n-1}): the new
        state solves x = r + beta h f(x) with r = a y_n - b y_{n-1}; the
        coefficients make the quadratic through the three states have slope
        f(x) at the new point. With w = h / h1: a = (1 + w)^2 / (1 + 2 w),
        b = w^2 / (1 + 2 w), beta = (1 + w) / (1 + 2 w)."""
        w = h / h1
        return (1 + w) ** 2 / (1 + 2 * w), w * w / (1 + 2 * w), (1 + w) / (1 + 2 * w)

    @staticmethod
    def bdf2_estimate_factor(h, h1, h2):
        """Local error of a BDF2 step from the gap between the corrector and
        the quadratic extrapolation of the last three states. Along the rule's
        own trajectory z the scheme's relation holds exactly, which makes z
        the solution of y' = f(y) + (z'''/6) h (h + h1); over the step that
        is a deviation of (1/6) h^2 (h + h1) y''' from the exact flow through
        the current state, while the extrapolation misses z(t + h) by
        (1/6) h (h + h1) (h + h1 + h2) y'''. Their ratio is h / (h + h1 + h2)."""
        return h / (h + h1 + h2)

    def implicit_bdf2_adaptive(self, m, t_end, dt0, alpha, lte_tol, method="aim",
                               terms=("ex", "ms"), h_app=None, tol=1e-13, max_newton=10,
                               A=None, max_steps=100000, record=False):
        """Time-step adaptive BDF2 (the paper's timed dynamics run uses a
        step-adaptive BDF scheme, Sec. 2.2 and Sec. 5; its formulas are this
        oracle's reading), a predictor-corrector pair like
        ``implicit_midpoint_adaptive``:

        * the first step is backward Euler (x = m + h f(x)) from the
          predictor m; the later ones BDF2 (``bdf2_coefficients``);
        * predictor: the line through the last two states (second step) or
          the quadratic through the last three, extrapolated to t + h;
        * corrector: Newton from the predictor (exact dense Jacobian of
          x - r - beta h f(x)), converged at residual rms <= tol; a failure
          halves the step;
        * from the third accepted step on, E = ``bdf2_estimate_factor`` times
          rms(x_c - x_p); E > lte_tol rejects the step; step control and the
          renormalisation of each accepted state as in the midpoint version.

        Returns (m, info) as ``implicit_midpoint_adaptive``; with ``record``,
        info["states"] holds the initial and every accepted state."""
        n = self.n
        A = self.field_matrix(method, terms) if A is None else A
        b = np.zeros(3) if h_app is None else np.asarray(h_app, dtype=np.float64)
        c = -GAMMA0 / (1 + alpha * alpha)
        m = np.array(m, dtype=np.float64, copy=True)
        rms = np.sqrt(3.0 * n)

        def newton(x, r, bh):
            g0 = None
            for it in range(max_newton + 1):
                H = (A @ x.ravel()).reshape(n, 3) + b[None, :]
                mxh = np.cross(x, H)
                G = x - r - bh * c * (mxh + alpha * np.cross(x, mxh))
                g = np.linalg.norm(G) / rms
                if g <= tol:
                    return x, it
                if it == max_newton or not np.isfinite(g) or (g0 is not None and g > 3 * g0):
                    return None, it
                g0 = g if g0 is None else g0
                CH, CM, CMH = self._cross_matrix(H), self._cross_matrix(x), self._cross_matrix(mxh)
                local = -CH - alpha * CMH - alpha * CM @ CH
                left = CM + alpha * CM @ CM
                J = np.zeros((3 * n, 3 * n))
                for k in range(n):
                    J[3 * k:3 * k + 3, 3 * k:3 * k + 3] += local[k]
                    J[3 * k:3 * k + 3, :] += left[k] @ A[3 * k:3 * k + 3, :]
                dG = np.eye(3 * n) - bh * c * J
                x = x - np.linalg.solve(dG, G.ravel()).reshape(n, 3)
            return None, max_newton

        t, dt = 0.0, float(dt0)
        hist = []                                    # [(state, step from it)], latest first
        info = dict(dts=[], lte=[], newton=[], rejected=0, dt_next=dt)
        if record:
            info["states"] = [m.copy()]
        while t_end - t > 1e-12 * t_end:
            if len(info["dts"]) >= max_steps:
                raise RuntimeError("adaptive BDF2: step limit")
            h = min(dt, t_end - t)
            if h < 1e-9 * t_end:
                raise RuntimeError("adaptive BDF2: time step underflow")
            if not hist:
                r, bh, xp = m, h, m.copy()
            else:
                y1, h1 = hist[0]
                a, bb, beta = self.bdf2_coefficients(h, h1)
                r, bh = a * m - bb * y1, beta * h
                if len(hist) >= 2:
                    y2, h2 = hist[1]
                    l0 = (h + h1) * (h + h1 + h2) / (h1 * (h1 + h2))
                    l1 = -h * (h + h1 + h2) / (h1 * h2)
                    l2 = h * (h + h1) / ((h1 + h2) * h2)
                    xp = l0 * m + l1 * y1 + l2 * y2
                else:
                    xp = m + (h / h1) * (m - y1)
            x, its = newton(xp.copy(), r, bh)
            if x is None:
                info["rejected"] += 1
                dt = 0.5 * h
                continue
            est = None
            dt_new = dt
            if len(hist) >= 2:
                est = self.bdf2_estimate_factor(h, hist[0][1], hist[1][1]) * \
                    np.linalg.norm(x - xp) / rms
                fac = 0.9 * (lte_tol / est) ** (1.0 / 3.0) if est > 0 else 2.0
                if est > lte_tol:
                    info["rejected"] += 1
                    dt = h * max(0.2, min(0.9, fac))
                    continue
                dt_new = h * min(2.0, max(0.2, fac))
            x = x / np.linalg.norm(x, axis=1, keepdims=True)
            # history: the earlier states, each with the step that leaves it
            hist.insert(0, (m, h))
            del hist[2:]
            m = x
            t += h
            if record:
                info["states"].append(m.copy())
            info["dts"].append(h)
            info["lte"].append(est)
            info["newton"].append(its)
            dt = dt_new
        info["dt_next"] = dt
        return m, info
