"""Multigrid pieces on the assembled hierarchy (oracle, test-only).

The paper builds geometric multigrid into the data structures (Section 5.1:
every function lives on a range of levels) but prints no transfer operators,
smoother parameters or coarse solver.  The readings used here:

* prolongation P: nested P1 interpolation.  Regular refinement makes the coarse
  P1 space a subspace of the fine one, so P is read off the refinement
  bookkeeping -- a fine vertex that coincides with a coarse vertex copies it
  (weight 1), a fine vertex created as the midpoint of a coarse micro-edge
  takes half of each endpoint (weights 1/2, 1/2);
* restriction R = P^T (unscaled), so R A_fine P = A_coarse;
* smoother: weighted Jacobi with omega = 2/3 (Section 5.2.1 names
  diagonal-based smoothers as the ones element-wise operators support);
* coarse solver: dense Cholesky of the interior coarse matrix;
* V(nu1, nu2) cycle in the textbook recursive form;
* optional Chebyshev smoother (the paper's large runs accelerate Jacobi with
  Chebyshev polynomials): the Chebyshev iteration for the Jacobi-
  preconditioned system D^-1 A u = D^-1 b on the interval [beta/8, beta],
  beta = 1.1 times an estimate of the largest eigenvalue of D^-1 A from 20
  power iterations started at sin(1000 x + 1700 y + 2300 z).  (A smoother
  only has to damp the upper part of the spectrum; with degree 2 the
  ratio 8 gives V(1,1) cycles contracting the residual by about 0.2.)
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .fem import P1System
from .refine import MicroMesh, keys_of


def prolongation(coarse: MicroMesh, fine: MicroMesh) -> sp.csr_matrix:
    """P from level l-1 to level l by refinement bookkeeping.

    Each coarse micro-tet of each macro-cell is refined once with eq. (bey);
    its 4 vertices map to themselves and its 6 edge midpoints to the mean of
    the edge's end points.  Entries met several times (shared edges) are the
    same and are kept once.
    """
    assert fine.level == coarse.level + 1
    T = len(coarse.local)
    W = coarse.local
    edges = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    rows, cols, vals = [], [], []
    for c in range(len(coarse.cells)):
        cidx = coarse.tets[c * T:(c + 1) * T]            # [T, 4]
        ids = coarse.cells[c]
        # vertices: fine weights are the coarse weights doubled
        for q in range(4):
            f = fine.index_of(keys_of(ids, 2 * W[:, q]))
            rows.append(f); cols.append(cidx[:, q]); vals.append(np.ones(T))
        # midpoints of the six edges
        for a, b in edges:
            f = fine.index_of(keys_of(ids, W[:, a] + W[:, b]))
            for e in (a, b):
                rows.append(f); cols.append(cidx[:, e])
                vals.append(np.full(T, 0.5))
    rows = np.concatenate(rows); cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    pair = rows.astype(np.int64) * coarse.num_vertices + cols
    _, first = np.unique(pair, return_index=True)
    P = sp.coo_matrix((vals[first], (rows[first], cols[first])),
                      shape=(fine.num_vertices, coarse.num_vertices)).tocsr()
    return P


# Chebyshev smoother parameters (readings, see the module docstring)
CHEB_PROBE = (1000.0, 1700.0, 2300.0)
CHEB_POWER_ITERS = 20
CHEB_UPPER = 1.1
CHEB_RATIO = 8.0


def lambda_max_estimate(S: P1System, iters: int = CHEB_POWER_ITERS) -> float:
    """Power iteration for the largest eigenvalue of D^-1 A on the interior
    unknowns: v <- D^-1 A v from the probe sin(k . x), estimate
    |v_new| / |v_old| of the last step (Euclidean norms)."""
    I = S.interior
    v = np.where(I, np.sin(S.mesh.xyz @ np.array(CHEB_PROBE)), 0.0)
    lam = 0.0
    for _ in range(iters):
        w = np.where(I, (S.A @ v) / S.diag, 0.0)
        lam = np.linalg.norm(w[I]) / np.linalg.norm(v[I])
        v = w
    return lam


def chebyshev_bounds(lam: float):
    """Smoothing interval [alpha, beta] from a largest-eigenvalue estimate."""
    beta = CHEB_UPPER * lam
    return beta / CHEB_RATIO, beta


def chebyshev_smooth(S: P1System, u: np.ndarray, b: np.ndarray, degree: int,
                     alpha: float, beta: float) -> np.ndarray:
    """One application of the degree-m Chebyshev iteration for
    D^-1 A u = D^-1 b on [alpha, beta] (the classical three-term form):
    theta = (beta + alpha)/2, delta = (beta - alpha)/2, sigma = theta/delta;
    d_0 = D^-1 r_0 / theta; then u_{k+1} = u_k + d_k and
    d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / delta) D^-1 r_k with
    rho_0 = 1/sigma, rho_k = 1/(2 sigma - rho_{k-1}).  The error of an
    eigenvector of D^-1 A with eigenvalue lam is multiplied by
    T_m((beta + alpha - 2 lam)/(beta - alpha)) / T_m((beta + alpha)/(beta - alpha)).
    Dirichlet values are kept."""
    I = S.interior
    theta, delta = 0.5 * (beta + alpha), 0.5 * (beta - alpha)
    sigma = theta / delta
    u = u.copy()
    d = np.zeros_like(u)
    rho_prev = rho = 1.0 / sigma
    for k in range(degree):
        z = np.where(I, (b - S.A @ u) / S.diag, 0.0)
        if k == 0:
            d = z / theta
        else:
            rho = 1.0 / (2.0 * sigma - rho_prev)
            d = rho * rho_prev * d + (2.0 * rho / delta) * z
            rho_prev = rho
        u = u + d
    return u


class Hierarchy:
    """Assembled systems on levels min_level..max_level plus transfers."""

    def __init__(self, xyz, cells, max_level: int, min_level: int = 0):
        self.min_level, self.max_level = int(min_level), int(max_level)
        self.sys = {}
        for lvl in range(self.min_level, self.max_level + 1):
            self.sys[lvl] = P1System(MicroMesh(xyz, cells, lvl))
        self.P = {}
        for lvl in range(self.min_level + 1, self.max_level + 1):
            self.P[lvl] = prolongation(self.sys[lvl - 1].mesh,
                                       self.sys[lvl].mesh)
        self._chol = {}
        self._cheb = {}

    def cheb_bounds(self, lvl: int):
        if lvl not in self._cheb:
            self._cheb[lvl] = chebyshev_bounds(lambda_max_estimate(self.sys[lvl]))
        return self._cheb[lvl]

    def smooth(self, lvl: int, u, b, sweeps: int, omega: float,
               smoother: str = "jacobi", degree: int = 2):
        """`sweeps` applications of the smoother on level lvl."""
        S = self.sys[lvl]
        if smoother == "jacobi":
            return S.jacobi(u, b, omega, sweeps)
        alpha, beta = self.cheb_bounds(lvl)
        for _ in range(sweeps):
            u = chebyshev_smooth(S, u, b, degree, alpha, beta)
        return u

    def __getitem__(self, lvl) -> P1System:
        return self.sys[lvl]

    # -- transfers --------------------------------------------------------
    def restrict(self, lvl: int, r: np.ndarray) -> np.ndarray:
        """R r = P^T r from level lvl to lvl-1 (fine Dirichlet entries of r
        are taken as zero, coarse Dirichlet entries are set to zero)."""
        r = np.where(self.sys[lvl].dirichlet, 0.0, r)
        rc = self.P[lvl].T @ r
        rc[self.sys[lvl - 1].dirichlet] = 0.0
        return rc

    def prolongate_add(self, lvl: int, e: np.ndarray, u: np.ndarray):
        """u + P e from level lvl to lvl+1 (coarse Dirichlet entries of e are
        taken as zero)."""
        e = np.where(self.sys[lvl].dirichlet, 0.0, e)
        return u + self.P[lvl + 1] @ e

    # -- coarse solve -----------------------------------------------------
    def coarse_solve(self, lvl: int, u: np.ndarray, b: np.ndarray):
        """Exact solve of the interior equations, Dirichlet values kept."""
        S = self.sys[lvl]
        I = np.flatnonzero(S.interior)
        if lvl not in self._chol:
            AII = S.A[I][:, I].toarray()
            self._chol[lvl] = sla.cho_factor(AII) if len(I) else None
        u = u.copy()
        if len(I) == 0:
            return u
        ub = np.where(S.dirichlet, u, 0.0)
        rhs = b[I] - (S.A @ ub)[I]
        u[I] = sla.cho_solve(self._chol[lvl], rhs)
        return u

    # -- cycles -----------------------------------------------------------
    def vcycle(self, lvl: int, u: np.ndarray, b: np.ndarray, nu1: int = 2,
               nu2: int = 2, omega: float = 2.0 / 3.0,
               coarse_level: int | None = None, smoother: str = "jacobi",
               degree: int = 2) -> np.ndarray:
        """One V(nu1, nu2) cycle for A u = b on level lvl (nu1, nu2 count
        smoother applications: Jacobi sweeps, or Chebyshev polynomials of
        the given degree)."""
        if coarse_level is None:
            coarse_level = self.min_level
        S = self.sys[lvl]
        if lvl == coarse_level:
            return self.coarse_solve(lvl, u, b)
        u = self.smooth(lvl, u, b, nu1, omega, smoother, degree)
        r = S.residual(u, b)
        bc = self.restrict(lvl, r)
        ec = np.zeros(self.sys[lvl - 1].mesh.num_vertices)
        ec = self.vcycle(lvl - 1, ec, bc, nu1, nu2, omega, coarse_level,
                         smoother, degree)
        u = self.prolongate_add(lvl - 1, ec, u)
        return self.smooth(lvl, u, b, nu2, omega, smoother, degree)

    def fmg(self, lvl: int, b: np.ndarray, cycles: int = 1, nu1: int = 2,
            nu2: int = 2, omega: float = 2.0 / 3.0,
            coarse_level: int | None = None) -> np.ndarray:
        """Full multigrid (nested iteration) for A u = b on level lvl with
        zero Dirichlet data: the right-hand side is carried down by the
        restriction (b_{l-1} = R b_l), the coarsest system is solved
        exactly, and on every finer level the interpolated coarser solution
        (P u_{l-1}) starts `cycles` V(nu1, nu2) cycles."""
        if coarse_level is None:
            coarse_level = self.min_level
        rhs = {lvl: b}
        for lv in range(lvl, coarse_level, -1):
            rhs[lv - 1] = self.restrict(lv, rhs[lv])
        u = self.coarse_solve(coarse_level,
                              np.zeros(self.sys[coarse_level].mesh.num_vertices),
                              rhs[coarse_level])
        for lv in range(coarse_level + 1, lvl + 1):
            u = self.prolongate_add(lv - 1, u,
                                    np.zeros(self.sys[lv].mesh.num_vertices))
            for _ in range(cycles):
                u = self.vcycle(lv, u, rhs[lv], nu1, nu2, omega, coarse_level)
        return u

    def solve(self, lvl: int, b: np.ndarray, u0: np.ndarray | None = None,
              rel_tol: float = 1e-10, max_cycles: int = 50, nu1: int = 2,
              nu2: int = 2, omega: float = 2.0 / 3.0,
              coarse_level: int | None = None):
        """V-cycles from u0 (default 0) until ||b - A u||_2 / ||b||_2 <= tol,
        both norms over interior vertices.  Returns (u, [relative residual
        before cycle 0, after cycle 1, ...])."""
        S = self.sys[lvl]
        u = np.zeros_like(b) if u0 is None else u0.copy()
        bnorm = np.linalg.norm(b[S.interior])
        hist = []
        for _ in range(max_cycles + 1):
            rel = np.linalg.norm(S.residual(u, b)) / bnorm
            hist.append(rel)
            if rel <= rel_tol or len(hist) > max_cycles:
                break
            u = self.vcycle(lvl, u, b, nu1, nu2, omega, coarse_level)
        return u, hist
