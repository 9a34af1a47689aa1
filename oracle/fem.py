"""Element-by-element P1 assembly on the explicit micro-mesh (oracle, test-only).

Section 5.2.1 of the paper: the stiffness entry a_ij is the sum over elements T
of the integral over T of grad(phi_i) . grad(phi_j); the element matrix of T
holds these integrals for its four vertex basis functions.  For P1 on a
straight tetrahedron the gradients are constant, so the integral is the
element volume times the dot product (exact, no quadrature choice involved).

Dirichlet boundary: a micro-face that belongs to exactly one micro-tet lies on
the domain boundary; its three vertices are Dirichlet vertices.  The rest are
the interior unknowns.

Lumped mass: m_i = sum over micro-tets T containing i of |T| / 4, the row sums
of the consistent P1 mass matrix.

Variable coefficient (Section 5.2.1, the div(k grad) element-wise operator of
the operator catalogue): a_ij = sum over T of the integral over T of
k grad(phi_i) . grad(phi_j).  The coefficient k is given by its values at the
micro-vertices and enters as its linear interpolant; the element integral of
k is taken with a degree-3 quadrature rule on the tetrahedron (the "q3" of the
form's name), exact for this integrand.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .refine import MicroMesh


def barycentric_gradients(P: np.ndarray):
    """Gradients of the four barycentric functions and the volume of every
    tet.  ``P``: [M, 4, 3] vertex coordinates.  Returns (G [M,4,3], vol [M]).

    With E the matrix whose rows are the edge vectors P_r - P_0 (r = 1..3),
    lambda_q (q >= 1) satisfies E grad(lambda_q) = e_q, hence grad(lambda_q)
    is column q of inv(E); grad(lambda_0) = -(sum of the other three).
    """
    E = P[:, 1:, :] - P[:, :1, :]
    Einv = np.linalg.inv(E)
    G = np.empty(P.shape, dtype=np.float64)
    G[:, 1:, :] = np.transpose(Einv, (0, 2, 1))
    G[:, 0, :] = -G[:, 1:, :].sum(axis=1)
    vol = np.abs(np.linalg.det(E)) / 6.0
    return G, vol


# Degree-3 rule on a tetrahedron: the centroid with weight -4/5 and the four
# points with barycentric coordinates (1/2, 1/6, 1/6, 1/6) and permutations,
# weight 9/20 each (weights relative to the volume; they sum to one).
TET_Q3_POINTS = np.array([[0.25, 0.25, 0.25, 0.25],
                          [0.5, 1 / 6, 1 / 6, 1 / 6],
                          [1 / 6, 0.5, 1 / 6, 1 / 6],
                          [1 / 6, 1 / 6, 0.5, 1 / 6],
                          [1 / 6, 1 / 6, 1 / 6, 0.5]])
TET_Q3_WEIGHTS = np.array([-0.8, 0.45, 0.45, 0.45, 0.45])


def element_coefficient_mean(kv: np.ndarray) -> np.ndarray:
    """(1/|T|) times the integral over T of the linear interpolant of k, by
    the degree-3 rule.  ``kv``: [M, 4] coefficient values at the vertices."""
    at_points = kv @ TET_Q3_POINTS.T          # [M, 5] k at the rule's points
    return at_points @ TET_Q3_WEIGHTS


def element_stiffness(P: np.ndarray):
    """Local stiffness matrices K_T[q, r] = |T| grad(l_q) . grad(l_r)."""
    G, vol = barycentric_gradients(P)
    K = vol[:, None, None] * np.einsum("mqd,mrd->mqr", G, G)
    return K, vol


class P1System:
    """Assembled P1 stiffness matrix of one micro-mesh, with boundary and
    mass: the Laplacian, or div(k grad) when ``kappa`` (values of k at the
    micro-vertices, canonical key order) is given."""

    def __init__(self, mesh: MicroMesh, kappa: np.ndarray | None = None):
        self.mesh = mesh
        N = mesh.num_vertices
        P = mesh.xyz[mesh.tets]
        K, vol = element_stiffness(P)
        if kappa is not None:
            K = K * element_coefficient_mean(kappa[mesh.tets])[:, None, None]
        rows = np.repeat(mesh.tets, 4, axis=1).ravel()
        cols = np.tile(mesh.tets, (1, 4)).ravel()
        self.A = sp.coo_matrix((K.ravel(), (rows, cols)),
                               shape=(N, N)).tocsr()
        self.A.sum_duplicates()
        self.tet_volume = vol
        self.lumped_mass = np.bincount(mesh.tets.ravel(),
                                       weights=np.repeat(vol / 4.0, 4),
                                       minlength=N)
        faces, counts = mesh.faces(return_counts=True)
        self.dirichlet = np.zeros(N, dtype=bool)
        self.dirichlet[faces[counts == 1].ravel()] = True
        self.interior = ~self.dirichlet
        self.diag = self.A.diagonal()

    # -- operators on full vectors (all vertices, canonical key order) ----
    def apply(self, x: np.ndarray) -> np.ndarray:
        """y_I = A_{I,:} x (boundary values of x act as Dirichlet data);
        y = 0 at Dirichlet vertices."""
        y = self.A @ x
        y[self.dirichlet] = 0.0
        return y

    def residual(self, u: np.ndarray, b: np.ndarray) -> np.ndarray:
        """r = b - A u on interior vertices, 0 at Dirichlet vertices."""
        r = b - self.A @ u
        r[self.dirichlet] = 0.0
        return r

    def jacobi(self, u: np.ndarray, b: np.ndarray, omega: float,
               sweeps: int = 1) -> np.ndarray:
        """Weighted Jacobi u <- u + omega D^-1 (b - A u) on interior vertices;
        Dirichlet values are kept."""
        u = u.copy()
        for _ in range(sweeps):
            r = b - self.A @ u
            u[self.interior] += omega * r[self.interior] / self.diag[self.interior]
        return u

    def interior_matrix(self):
        I = np.flatnonzero(self.interior)
        return self.A[I][:, I], I
