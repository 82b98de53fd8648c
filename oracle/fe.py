"""P1 finite elements for the 2-D eddy-current A-formulation (oracle, FP64).

Paper, Section 2, eq. (1): ``M du/dt + K(u) u = f(t)`` with M the singular
conductivity matrix, K(u) the (nonlinear) curl-curl matrix and f the excitation.
The paper names only "the finite element method" (Section 4); the reading taken
here is linear (P1) triangles, the exact (consistent) conductivity mass
``M_e = sigma_e*A_e/12*(1 + delta_ij)`` and the load ``F_e,i = js_e*A_e/3``.
In 2-D, ``B = curl(A e_z)`` so ``|B|^2 = |grad A|^2``; per element
``|grad A_h|^2 = u_e^T K0_e u_e / A_e`` with ``K0_e,ij = (b_i b_j + c_i c_j)/(4 A_e)``.

TEST INFRASTRUCTURE ONLY: see the package docstring.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

LINEAR = 0
BRAUER = 1


def element_geometry(xy, tri):
    """Edge coefficients b_i = y_{i+1}-y_{i+2}, c_i = x_{i+2}-x_{i+1} (cyclic) and |area|."""
    x = xy[tri, 0]
    y = xy[tri, 1]
    b = np.stack([y[:, 1] - y[:, 2], y[:, 2] - y[:, 0], y[:, 0] - y[:, 1]], axis=1)
    c = np.stack([x[:, 2] - x[:, 1], x[:, 0] - x[:, 2], x[:, 1] - x[:, 0]], axis=1)
    area = 0.5 * np.abs(b[:, 0] * c[:, 1] - b[:, 1] * c[:, 0])
    return b, c, area


def unit_stiffness(b, c, area):
    """K0_e (n_e x 3 x 3): the curl-curl element matrix for unit reluctivity."""
    return (b[:, :, None] * b[:, None, :] + c[:, :, None] * c[:, None, :]) / (4.0 * area[:, None, None])


def element_mass(sigma, area):
    """Consistent conductivity mass sigma*A/12*(1+delta_ij)."""
    base = (np.ones((3, 3)) + np.eye(3)) / 12.0
    return (sigma * area)[:, None, None] * base[None, :, :]


def reluctivity(b2, model, par):
    """nu(b2) and dnu/d(b2) per element for the material of that element.

    Linear: nu = par[0].  Brauer: nu = k1*exp(k2*b2) + k3 (par = nu, k1, k2, k3)."""
    nu = np.where(model == LINEAR, par[:, 0], 0.0).astype(np.float64)
    dnu = np.zeros_like(nu)
    br = model == BRAUER
    if np.any(br):
        e = np.exp(par[br, 2] * b2[br])
        nu[br] = par[br, 1] * e + par[br, 3]
        dnu[br] = par[br, 1] * par[br, 2] * e
    return nu, dnu


class FE:
    """Discrete operators of eq. (1) on the free (non-Dirichlet) nodes."""

    def __init__(self, prob):
        self.prob = prob
        n_nodes = prob.xy.shape[0]
        self.n_nodes = n_nodes
        self.tri = prob.tri.astype(np.int64)
        b, c, area = element_geometry(prob.xy, prob.tri)
        self.b, self.c, self.area = b, c, area
        self.K0 = unit_stiffness(b, c, area)
        self.Me = element_mass(prob.sigma, area)
        self.model = prob.mat_model[prob.mat_id]
        self.par = prob.mat_par[prob.mat_id]
        is_dir = np.zeros(n_nodes, dtype=bool)
        is_dir[prob.dirichlet] = True
        self.free = np.flatnonzero(~is_dir)
        self.n = len(self.free)
        # restriction: full node vector -> free vector
        self.R = sp.csr_matrix((np.ones(self.n), (np.arange(self.n), self.free)),
                               shape=(self.n, n_nodes))
        self.M = self._restrict(self.assemble(self.Me))
        load = (prob.js * area / 3.0)[:, None] * np.ones((1, 3))
        Ffull = np.zeros(n_nodes)
        np.add.at(Ffull, self.tri, load)
        self.F = Ffull[self.free]

    # -- assembly helpers --------------------------------------------------------------
    def assemble(self, Ke):
        rows = np.repeat(self.tri, 3, axis=1).ravel()
        cols = np.tile(self.tri, (1, 3)).ravel()
        return sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(self.n_nodes, self.n_nodes))

    def _restrict(self, A):
        return (self.R @ A @ self.R.T).tocsr()

    def full(self, u):
        """Free vector(s) -> nodal vector(s) with A = 0 on the Dirichlet ring."""
        u = np.asarray(u)
        out = np.zeros(u.shape[:-1] + (self.n_nodes,), dtype=u.dtype)
        out[..., self.free] = u
        return out

    def f(self, t):
        """Excitation vector f(t) = i(t) F (eq. 1)."""
        return float(self.prob.current(t)) * self.F

    # -- nonlinear curl-curl ------------------------------------------------------------
    def element_state(self, u):
        """Per-element w = K0_e u_e, b2 = |grad A_h|^2, nu, dnu at the free vector u."""
        ue = self.full(u)[self.tri]
        w = np.einsum("eij,ej->ei", self.K0, ue)
        b2 = np.einsum("ei,ei->e", ue, w) / self.area
        nu, dnu = reluctivity(b2, self.model, self.par)
        return ue, w, b2, nu, dnu

    def K_apply(self, u):
        """K(u) u = sum_e nu(|grad A|^2) K0_e u_e (free rows)."""
        _, w, _, nu, _ = self.element_state(u)
        out = np.zeros(self.n_nodes)
        np.add.at(out, self.tri, nu[:, None] * w)
        return out[self.free]

    def K_matrix(self, nu):
        """Sum_e nu_e K0_e for given per-element reluctivities (free block)."""
        return self._restrict(self.assemble(nu[:, None, None] * self.K0))

    def jacobian_curl(self, u):
        """d(K(u)u)/du = sum_e [nu K0_e + (2 nu'/A_e)(K0_e u)(K0_e u)^T]."""
        _, w, _, nu, dnu = self.element_state(u)
        Ke = nu[:, None, None] * self.K0 + (2.0 * dnu / self.area)[:, None, None] * (
            w[:, :, None] * w[:, None, :])
        return self._restrict(self.assemble(Ke))

    def linearised_stiffness(self, U):
        """Frozen time-averaged linearisation over coarse samples U (rows = samples).

        Reading of the nonlinear coarse treatment that the paper defers (Section 2,
        after eq. (10)): per element, average the differential reluctivity tensor
        ``nu I + 2 nu' g g^T`` (g = grad A_h) over the samples, then
        ``Kbar_e = A_e G_e nubar_e G_e^T`` with G_e the 3x2 matrix of basis gradients.
        For a linear material this is nu K0_e exactly."""
        U = np.atleast_2d(U)
        Gx = self.b / (2.0 * self.area[:, None])     # d phi_i/dx (sign of area cancels below)
        Gy = self.c / (2.0 * self.area[:, None])
        sgn = np.sign(self.b[:, 0] * self.c[:, 1] - self.b[:, 1] * self.c[:, 0])
        Gx = Gx * sgn[:, None]
        Gy = Gy * sgn[:, None]
        nxx = np.zeros(len(self.area))
        nxy = np.zeros(len(self.area))
        nyy = np.zeros(len(self.area))
        for u in U:
            ue = self.full(u)[self.tri]
            gx = np.einsum("ei,ei->e", Gx, ue)
            gy = np.einsum("ei,ei->e", Gy, ue)
            nu, dnu = reluctivity(gx * gx + gy * gy, self.model, self.par)
            nxx += nu + 2.0 * dnu * gx * gx
            nxy += 2.0 * dnu * gx * gy
            nyy += nu + 2.0 * dnu * gy * gy
        nxx /= len(U)
        nxy /= len(U)
        nyy /= len(U)
        Ke = self.area[:, None, None] * (
            nxx[:, None, None] * Gx[:, :, None] * Gx[:, None, :]
            + nxy[:, None, None] * (Gx[:, :, None] * Gy[:, None, :] + Gy[:, :, None] * Gx[:, None, :])
            + nyy[:, None, None] * Gy[:, :, None] * Gy[:, None, :])
        return self._restrict(self.assemble(Ke))
