"""Pins of the oracle's P1 finite elements (Section 2, eq. (1); Section 4 "finite element
method") against mesh geometry, closed-form element matrices and finite differences."""
import math

import numpy as np
import pytest

from oracle.fe import FE, element_geometry, reluctivity, unit_stiffness
from oracle.timestep import step_residual
from workloads import coax


def test_mesh_counts_and_ring_layout():
    # structured polar mesh: 1 + nr*ntheta nodes, ntheta*(2 nr - 1) triangles
    for gen, nr, nt, rings in [(coax.c1, 20, 40, [7, 7, 3, 3]), (coax.c2, 60, 120, [20, 20, 10, 10])]:
        p = gen()
        assert p.n_nodes == 1 + nr * nt
        assert p.n_tri == nt * (2 * nr - 1)
        assert len(p.dirichlet) == nt
        assert p.meta["ring_counts"] == rings
    # the large workload's ring split (no FE assembly needed)
    assert coax.ring_counts([1, 1, 0.5, 0.5], 400).tolist() == [133, 133, 67, 67]


@pytest.mark.parametrize("gen", [coax.c1, coax.c2])
def test_total_area_is_inscribed_polygon(gen):
    p = gen()
    _, _, area = element_geometry(p.xy, p.tri)
    R, nt = 3e-3, p.meta["ntheta"]
    exact = 0.5 * nt * R * R * math.sin(2 * math.pi / nt)
    assert abs(area.sum() - exact) <= 1e-14 * exact


def test_structural_nnz_matches_edge_count():
    # free-free couplings of the polar mesh: n_free + 2 * ntheta (3 nr - 4)
    for gen, nr, nt in [(coax.c1, 20, 40), (coax.c2, 60, 120)]:
        fe = FE(gen())
        ones = fe._restrict(fe.assemble(np.ones((fe.prob.n_tri, 3, 3))))
        assert ones.nnz == fe.n + 2 * nt * (3 * nr - 4)


def test_source_density_gives_exact_net_currents():
    p = coax.c1()
    _, _, area = element_geometry(p.xy, p.tri)
    core = p.js > 0
    outer = p.js < 0
    assert abs((p.js[core] * area[core]).sum() - 1.0) <= 1e-13
    assert abs((p.js[outer] * area[outer]).sum() + 1.0) <= 1e-13


def test_unit_stiffness_reference_triangle_and_row_sums():
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    tri = np.array([[0, 1, 2]])
    b, c, a = element_geometry(xy, tri)
    K0 = unit_stiffness(b, c, a)[0]
    np.testing.assert_allclose(K0, 0.5 * np.array([[2, -1, -1], [-1, 1, 0], [-1, 0, 1]]), atol=1e-15)
    # orientation does not matter
    b2, c2, a2 = element_geometry(xy, tri[:, ::-1])
    np.testing.assert_allclose(unit_stiffness(b2, c2, a2)[0], K0[::-1, ::-1], atol=1e-15)
    # translation invariance on a real mesh: every row sums to zero
    fe = FE(coax.c1())
    rs = np.abs(fe.K0.sum(axis=2)).max() / np.abs(fe.K0).max()
    assert rs <= 1e-13
    # symmetric positive semidefinite with the constant in the kernel
    ev = np.linalg.eigvalsh(fe.K0[:50])
    assert ev.min() >= -1e-10 * ev.max()


def test_conductivity_mass_sums_to_sigma_area():
    fe = FE(coax.c1())
    Mfull = fe.assemble(fe.Me)
    assert abs(Mfull.sum() - (fe.prob.sigma * fe.area).sum()) <= 1e-13 * (fe.prob.sigma * fe.area).sum()
    # M is singular: zero rows exactly on nodes touching only non-conducting elements
    rows = np.asarray(np.abs(fe.M).sum(axis=1)).ravel()
    assert (rows == 0).sum() > 0


def test_gradient_energy_identity():
    # u^T K0 u / A = |grad u_h|^2 for a linear field u = g . x
    fe = FE(coax.c2())
    g = np.array([3.0, -2.0])
    u = fe.prob.xy @ g
    ue = u[fe.tri]
    b2 = np.einsum("ei,eij,ej->e", ue, fe.K0, ue) / fe.area
    np.testing.assert_allclose(b2, g @ g, rtol=1e-9)


def test_brauer_law_values_and_derivative():
    model = np.array([1, 1, 1])
    par = np.array([[0.0, 3.8, 2.17, 396.2]] * 3)
    b2 = np.array([0.0, 1.0, 3.5])
    nu, dnu = reluctivity(b2, model, par)
    assert nu[0] == pytest.approx(3.8 + 396.2, rel=0, abs=1e-12)
    np.testing.assert_allclose(nu, 3.8 * np.exp(2.17 * b2) + 396.2, rtol=1e-15)
    h = 1e-6
    fd = (reluctivity(b2 + h, model, par)[0] - reluctivity(b2 - h, model, par)[0]) / (2 * h)
    np.testing.assert_allclose(dnu, fd, rtol=1e-7)
    lin, dl = reluctivity(b2, np.zeros(3, int), np.array([[coax.NU0, 0, 0, 0]] * 3))
    assert np.all(lin == coax.NU0) and np.all(dl == 0)


def _saturated_state(fe, scale=3e-3):
    # a field that drives the steel into saturation (|B| ~ 1-3 T)
    r = np.hypot(fe.prob.xy[:, 0], fe.prob.xy[:, 1])[fe.free]
    return scale * (3e-3 - r) / 3e-3 + 1e-5 * np.sin(7 * np.arctan2(fe.prob.xy[fe.free, 1], fe.prob.xy[fe.free, 0]))


def test_jacobian_matches_central_differences():
    prob = coax.tiny(nr=6, ntheta=12, nonlinear=True)
    fe = FE(prob)
    u = _saturated_state(fe)
    _, _, b2, _, _ = fe.element_state(u)
    assert np.sqrt(b2.max()) > 1.0          # nonlinear regime exercised
    dt = 1e-5
    up = 0.9 * u
    J = fe.M / dt + fe.jacobian_curl(u)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(fe.n) * 1e-3 * np.abs(u).max()
    h = 1e-6
    fd = (step_residual(fe, u + h * v, up, 0.003, dt) - step_residual(fe, u - h * v, up, 0.003, dt)) / (2 * h)
    assert np.linalg.norm(J @ v - fd) <= 1e-7 * np.linalg.norm(fd)


def test_linearised_stiffness_special_cases():
    prob = coax.tiny(nr=6, ntheta=12, nonlinear=True)
    fe = FE(prob)
    u = _saturated_state(fe)
    # one sample: the time-averaged differential tensor is the Jacobian's curl part
    Kb = fe.linearised_stiffness(u[None, :])
    Jc = fe.jacobian_curl(u)
    assert abs(Kb - Jc).max() <= 1e-11 * abs(Jc).max()
    # two identical samples give the same average
    Kb2 = fe.linearised_stiffness(np.stack([u, u]))
    assert abs(Kb2 - Kb).max() <= 1e-12 * abs(Kb).max()
    # all-linear materials: exactly nu K0
    fl = FE(coax.c1())
    Kl = fl.linearised_stiffness(np.zeros((2, fl.n)))
    K = fl.K_matrix(np.full(fl.prob.n_tri, coax.NU0))
    assert abs(Kl - K).max() <= 1e-12 * abs(K).max()
