"""The seeded synthetic workloads: mesh sizes of the configurations, mesh validity, exact
discrete source currents, the parameter ranges each generator draws from, and determinism.
These inputs stand in for the paper's coax (Section 4), whose geometry and B-H data are not
given."""
import numpy as np
import pytest

from workloads import coax


def _areas(prob):
    p = prob.xy[prob.tri]
    return 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) -
                  (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))


@pytest.mark.parametrize("make,nodes,free,tri", [(coax.c1, 801, 761, 1560), (coax.c2, 7201, 7081, 14280)])
def test_configuration_sizes(make, nodes, free, tri):
    prob = make()
    assert prob.n_nodes == nodes and prob.n_tri == tri
    assert prob.n_nodes - len(prob.dirichlet) == free


def test_c2_pattern_has_the_stated_entries():
    """CSR entries among the free nodes: the diagonal plus both directions of every mesh edge
    joining two free nodes."""
    prob = coax.c2()
    free = np.ones(prob.n_nodes, dtype=bool)
    free[prob.dirichlet] = False
    e = np.concatenate([prob.tri[:, [0, 1]], prob.tri[:, [1, 2]], prob.tri[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    e = e[free[e[:, 0]] & free[e[:, 1]]]
    assert int(free.sum()) + 2 * len(e) == 49321


def test_large_coax_sizes_and_excitation():
    prob = coax.c3()
    assert prob.n_nodes == 320001 and prob.n_tri == 639200
    assert prob.n_nodes - len(prob.dirichlet) == 319201
    assert (prob.N, prob.m) == (200, 100)
    assert list(prob.orders) == [1, 3]
    assert prob.amps[1] == pytest.approx(0.2 * prob.amps[0]) and 200.0 <= prob.amps[0] <= 800.0
    assert 0.0 <= prob.phases[1] < 2.0 * np.pi


@pytest.mark.parametrize("make", [coax.c1, coax.c2, coax.c5_small, lambda: coax.tiny(nonlinear=True)])
def test_meshes_are_valid(make):
    prob = make()
    assert np.all(_areas(prob) > 0.0)                       # counter-clockwise, none degenerate
    r = np.hypot(prob.xy[:, 0], prob.xy[:, 1])
    np.testing.assert_allclose(r[prob.dirichlet], r.max(), rtol=1e-12)   # the outer ring
    used = np.zeros(prob.n_nodes, dtype=bool)
    used[prob.tri.ravel()] = True
    assert used.all()
    # layer interfaces fall on rings
    radii = np.unique(np.round(r, 12))
    for ri in prob.meta["interfaces"]:
        assert np.min(np.abs(radii - ri)) < 1e-12


def test_discrete_source_currents_are_exact():
    """Each driven region carries +-1 A per ampere of i(t) on the discrete mesh (reading R12):
    the core in every configuration, plus the return in the outer conductor of C1."""
    for prob, want_total in ((coax.c1(), 0.0), (coax.c2(), 1.0), (coax.c5_small(), 1.0)):
        a = _areas(prob)
        core = prob.js > 0
        assert np.sum(prob.js[core] * a[core]) == pytest.approx(1.0, rel=1e-12)
        assert np.sum(prob.js * a) == pytest.approx(want_total, abs=1e-12)


def test_c2_amplitude_is_seeded_and_in_range():
    a = coax.c2()
    b = coax.c2()
    assert 200.0 <= a.amps[0] <= 800.0
    assert a.amps[0] == b.amps[0]
    np.testing.assert_array_equal(a.xy, b.xy)
    np.testing.assert_array_equal(a.tri, b.tri)
    assert coax.c2(seed=7).amps[0] != a.amps[0]


def test_batched_designs_draw_within_their_ranges():
    """The first designs of the 256-design batch (the draws are sequential, so they are the
    batch's own): nr in [20, 200], ntheta = 2 nr, sheath 0.2-1.0 mm, sheath conductivity in
    [1e5, 1e7] S/m, Brauer k2 in [1.5, 3.0], amplitude in [100, 800] A, N = 40 x 50."""
    designs = coax.c4_designs(n_designs=6)
    again = coax.c4_designs(n_designs=6)
    for d, e in zip(designs, again):
        nr, nt = d.meta["nr"], d.meta["ntheta"]
        assert 20 <= nr <= 200 and nt == 2 * nr
        assert 0.2e-3 <= d.meta["sheath"] <= 1.0e-3
        steel = d.mat_id == 1
        sig = np.unique(d.sigma[steel])
        assert len(sig) == 1 and 1e5 <= sig[0] <= 1e7
        assert 1.5 <= d.mat_par[1, 2] <= 3.0
        assert 100.0 <= d.amps[0] <= 800.0
        assert (d.N, d.m) == (40, 50)
        assert d.amps[0] == e.amps[0] and d.meta["nr"] == e.meta["nr"]


def test_parity_inputs_are_seeded():
    prob = coax.c2(nr=20, ntheta=40, N=4, m=2)
    free = np.setdiff1d(np.arange(prob.n_nodes), prob.dirichlet)
    a = coax.chain_starts(prob, free, seed=3)
    assert a.shape == (4, len(free))
    np.testing.assert_array_equal(a, coax.chain_starts(prob, free, seed=3))
    assert np.all(a >= 0.0)                       # a profile that vanishes on the outer ring
    rr = coax.random_rows(3, 10, seed=5, amp=2.0)
    np.testing.assert_array_equal(rr, coax.random_rows(3, 10, seed=5, amp=2.0))
    idx = coax.sample_index(1000, 50, seed=9)
    assert idx[0] == 0 and len(idx) == 50 and np.all(np.diff(idx) > 0) and idx[-1] < 1000
