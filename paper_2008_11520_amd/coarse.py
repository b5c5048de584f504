"""Coarse-level Navier-Stokes solver of the closed DNN-MG loop.

The coarse part of Algorithm 2 of the paper: at every time step the coarse velocity
and pressure (v_n, p_n) on level L are found by Newton's method for the
discrete problem, whose right-hand side is the restricted fine right-hand
side b_L of the previous step (its restriction).  Here, as in the fine step:

* Q1 velocity and Q1 pressure on a structured quadrilateral mesh (possibly
  perturbed; bilinear element maps), 2 x 2 Gauss quadrature;
* the theta scheme:  (1/dt) M v + theta (C(v) v + nu K v) - B^T p = b_L
  (momentum rows at nodes without a Dirichlet condition; v = v_D at the
  others), theta = 1 implicit Euler (Eq. (nonlinearshort) read for implicit
  Euler), theta = 1/2 Crank-Nicolson (Eq. (4cranknicholson3), no body force);
  the matrices are those of the fine defect.  The explicit part of the
  theta scheme, -(1 - theta) (C(u) u + nu K u) of the previous velocity u,
  belongs to the right-hand side (rhs_of);
* continuity with local projection stabilisation (Sec. 3.1), in its
  two-level form for equal-order Q1:
  (div v, xi) + sum_P alpha_P (grad p - k_P(grad p), grad xi - k_P(grad xi)) = 0,
  P the patches of 2 x 2 elements (a trailing odd row or column of elements
  joins the last patch), k_P the mean over the patch (projection onto
  constants on the patch), alpha_P = alpha0 h_P^2 / nu (Re = 1/nu),
  alpha0 = 0.1, h_P = sqrt(|P|) / 2.  The fluctuation vanishes for linear
  pressures and, unlike a per-element mean, does not vanish for a pressure
  that alternates from one element column (or row) to the next;
* Newton's method (Eq. (newton)) with the analytic Jacobian of the
  convection, C(v) w + C(w) v; each linear system is solved by a sparse LU
  factorisation (the paper uses GMRES with a multigrid preconditioner; this
  solver is not the optimisation target and runs on the host).

With no Dirichlet-free side the pressure is fixed by p = 0 at node 0 (its
continuity row is replaced); a constant pressure has no effect on the step.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_G = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))


class CoarseNS:
    """Q1/Q1 Navier-Stokes with the theta scheme on one structured mesh level.

    cxy: (ny+1, nx+1, 2) node coordinates (node (i, j) at index j (nx+1) + i);
    dirichlet: DNNMG_DIR_* side bits (others are do-nothing outflow);
    theta: 1 implicit Euler, 1/2 Crank-Nicolson."""

    def __init__(self, cxy, dt, nu, dirichlet, alpha0=0.1, theta=1.0):
        cxy = np.asarray(cxy, dtype=np.float64)
        self.ny, self.nx = cxy.shape[0] - 1, cxy.shape[1] - 1
        nx, ny = self.nx, self.ny
        self.N = (nx + 1) * (ny + 1)
        self.dt, self.nu, self.alpha0 = float(dt), float(nu), float(alpha0)
        self.theta = float(theta)
        xy = cxy.reshape(-1, 2)
        i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
        n00 = (j * (nx + 1) + i).reshape(-1)
        self.en = np.stack([n00, n00 + 1, n00 + nx + 1, n00 + nx + 2], axis=1)   # corners 00, 10, 01, 11
        E = self.en.shape[0]
        # per element and Gauss point: shape values, physical gradients, weight |det| / 4
        self.Nq = np.zeros((4, 4))                 # [q, a]
        self.dx = np.zeros((E, 4, 4))              # [e, q, a]
        self.dy = np.zeros((E, 4, 4))
        self.wd = np.zeros((E, 4))
        X, Y = xy[self.en, 0], xy[self.en, 1]      # (E, 4)
        q = 0
        for t in _G:
            for s in _G:
                N = np.array([(1 - s) * (1 - t), s * (1 - t), (1 - s) * t, s * t])
                Ns = np.array([-(1 - t), 1 - t, -t, t])
                Nt = np.array([-(1 - s), -s, 1 - s, s])
                xs, xt, ys, yt = X @ Ns, X @ Nt, Y @ Ns, Y @ Nt
                det = xs * yt - xt * ys
                if np.any(det <= 0):
                    raise ValueError("coarse mesh has an element that is not positively oriented")
                self.Nq[q] = N
                self.dx[:, q] = (yt[:, None] * Ns - ys[:, None] * Nt) / det[:, None]
                self.dy[:, q] = (-xt[:, None] * Ns + xs[:, None] * Nt) / det[:, None]
                self.wd[:, q] = 0.25 * det
                q += 1
        # Dirichlet nodes
        I = np.arange(self.N) % (nx + 1)
        J = np.arange(self.N) // (nx + 1)
        d = dirichlet
        self.dmask = (((d & 1) != 0) & (I == 0)) | (((d & 2) != 0) & (I == nx)) | \
                     (((d & 4) != 0) & (J == 0)) | (((d & 8) != 0) & (J == ny))
        self.pin_pressure = bool(d == 15)
        # constant matrices
        wN = self.wd[:, :, None, None] * self.Nq[None, :, :, None] * self.Nq[None, :, None, :]   # (E, q, a, b)
        self.M = self._assemble(wN.sum(1))
        gg = self.dx[:, :, :, None] * self.dx[:, :, None, :] + self.dy[:, :, :, None] * self.dy[:, :, None, :]
        Kloc = (self.wd[:, :, None, None] * gg).sum(1)
        self.K = self._assemble(Kloc)
        # G_c[a, k] = sum_q wd N_k d_c N_a: momentum row a, pressure column k
        self.Gx = self._assemble((self.wd[:, :, None, None] * self.dx[:, :, :, None] * self.Nq[None, :, None, :]).sum(1))
        self.Gy = self._assemble((self.wd[:, :, None, None] * self.dy[:, :, :, None] * self.Nq[None, :, None, :]).sum(1))
        # local projection stabilisation on 2 x 2-element patches:
        # S = sum_P alpha_P (sum_{T in P} K_T - g_P g_P^T / |P|), g_P the patch
        # integrals of the shape gradients
        px, py = max(nx // 2, 1), max(ny // 2, 1)
        pe = (np.minimum(j // 2, py - 1) * px + np.minimum(i // 2, px - 1)).reshape(-1)   # patch of each element
        NP = px * py
        area_e = self.wd.sum(1)
        area_p = np.bincount(pe, weights=area_e, minlength=NP)
        alpha_p = self.alpha0 * (area_p / 4.0) / self.nu
        self.S = self._assemble(alpha_p[pe][:, None, None] * Kloc)
        gx = (self.wd[:, :, None] * self.dx).sum(1)      # (E, a): int_T dN_a/dx
        gy = (self.wd[:, :, None] * self.dy).sum(1)
        for g in (gx, gy):
            Gp = sp.csr_matrix((g.reshape(-1), (np.repeat(pe, 4), self.en.reshape(-1))), shape=(NP, self.N))
            self.S = self.S - Gp.T @ sp.diags(alpha_p / area_p) @ Gp
        self.S = self.S.tocsr()

    def _assemble(self, loc):
        """Sum element matrices loc (E, 4, 4) [row node a, column node b]."""
        rows = np.repeat(self.en, 4, axis=1).reshape(-1)
        cols = np.tile(self.en, (1, 4)).reshape(-1)
        return sp.csr_matrix((loc.reshape(-1), (rows, cols)), shape=(self.N, self.N))

    def _convection(self, v):
        """C(v) (the operator u -> (v.grad u, phi)) and the two blocks of
        u -> (u.grad v_c, phi) for c = x, y, as (N x N) matrices."""
        vq = np.einsum("qa,eac->eqc", self.Nq, v[self.en])                  # (E, q, 2)
        adv = vq[:, :, 0, None] * self.dx + vq[:, :, 1, None] * self.dy     # (E, q, b): v.grad N_b
        C = self._assemble((self.wd[:, :, None, None] * self.Nq[None, :, :, None] * adv[:, :, None, :]).sum(1))
        ve = v[self.en]                                                      # (E, b, 2)
        dvx = np.einsum("eqb,ebc->eqc", self.dx, ve)                         # d v_c / dx at q
        dvy = np.einsum("eqb,ebc->eqc", self.dy, ve)
        NN = self.wd[:, :, None, None] * self.Nq[None, :, :, None] * self.Nq[None, :, None, :]   # (E, q, a, b)
        # (u.grad v)_c = u_x d_x v_c + u_y d_y v_c
        D = {(c, cp): self._assemble((NN * (dvx if cp == 0 else dvy)[:, :, c, None, None]).sum(1))
             for c in range(2) for cp in range(2)}
        return C, D

    def residual(self, v, p, b, vD):
        """Momentum (2N) and continuity (N) residual of A(v, p) - b, with the
        Dirichlet rows v - v_D and, when pinned, p_0."""
        C, _ = self._convection(v)
        A = self.M / self.dt + self.theta * (C + self.nu * self.K)
        r = np.empty(3 * self.N)
        r[:self.N] = A @ v[:, 0] - self.Gx @ p - b[:, 0]
        r[self.N:2 * self.N] = A @ v[:, 1] - self.Gy @ p - b[:, 1]
        r[2 * self.N:] = self.Gx.T @ v[:, 0] + self.Gy.T @ v[:, 1] + self.S @ p
        m = self.dmask
        r[:self.N][m] = v[m, 0] - vD[m, 0]
        r[self.N:2 * self.N][m] = v[m, 1] - vD[m, 1]
        if self.pin_pressure:
            r[2 * self.N] = p[0]
        return r

    def jacobian(self, v):
        C, D = self._convection(v)
        th = self.theta
        A = self.M / self.dt + th * (C + self.nu * self.K)
        J = sp.bmat([[A + th * D[0, 0], th * D[0, 1], -self.Gx],
                     [th * D[1, 0], A + th * D[1, 1], -self.Gy],
                     [self.Gx.T, self.Gy.T, self.S]], format="lil")
        rows = np.concatenate([np.flatnonzero(self.dmask), self.N + np.flatnonzero(self.dmask)])
        if self.pin_pressure:
            rows = np.concatenate([rows, [2 * self.N]])
        J = J.tocsr()
        # identity rows for the Dirichlet values (and the pinned pressure)
        keep = np.ones(3 * self.N)
        keep[rows] = 0.0
        J = sp.diags(keep) @ J + sp.csr_matrix((np.ones(rows.size), (rows, rows)), shape=J.shape)
        return J.tocsc()

    def solve(self, b, vD, v0, p0, tol=1e-11, max_newton=20):
        """Newton's method for A(v, p) = b from (v0, p0) with the Dirichlet
        values vD (N x 2).  Returns v (N x 2), p (N), Newton steps."""
        v = np.array(v0, dtype=np.float64).reshape(self.N, 2).copy()
        p = np.array(p0, dtype=np.float64).reshape(self.N).copy()
        b = np.asarray(b, dtype=np.float64).reshape(self.N, 2)
        vD = np.asarray(vD, dtype=np.float64).reshape(self.N, 2)
        r = self.residual(v, p, b, vD)
        # converged: residual below tol relative to the larger of the initial
        # residual, the right-hand side and the Dirichlet data
        scale = max(np.linalg.norm(r), np.linalg.norm(b), np.linalg.norm(vD), 1e-300)
        for it in range(max_newton):
            if np.linalg.norm(r) <= tol * scale:
                return v, p, it
            dx = spla.splu(self.jacobian(v)).solve(-r)
            v[:, 0] += dx[:self.N]
            v[:, 1] += dx[self.N:2 * self.N]
            p += dx[2 * self.N:]
            r = self.residual(v, p, b, vD)
        if np.linalg.norm(r) > tol * scale:
            raise RuntimeError("Newton did not converge: |r| = %.3e (scale %.3e)" % (np.linalg.norm(r), scale))
        return v, p, max_newton

    def mass_rhs(self, u):
        """(1/dt) M u: the implicit-Euler right-hand side of a velocity u on
        this level (the step without a network correction)."""
        u = np.asarray(u, dtype=np.float64).reshape(self.N, 2)
        return np.stack([self.M @ u[:, 0], self.M @ u[:, 1]], axis=1) / self.dt

    def transport(self, u):
        """T(u) = C(u) u + nu K u on this level (N x 2)."""
        u = np.asarray(u, dtype=np.float64).reshape(self.N, 2)
        C, _ = self._convection(u)
        A = C + self.nu * self.K
        return np.stack([A @ u[:, 0], A @ u[:, 1]], axis=1)

    def rhs_of(self, u):
        """The theta scheme's right-hand side of a previous velocity u on this
        level, (1/dt) M u - (1 - theta) T(u) (the step without a network
        correction)."""
        b = self.mass_rhs(u)
        if self.theta != 1.0:
            b = b - (1.0 - self.theta) * self.transport(u)
        return b
