"""Seeded synthetic coaxial-cable workloads for the periodic eddy-current problem.

This module only *generates inputs*: node coordinates, triangles, the Dirichlet
set, per-element material data, the per-unit-current source density and the
excitation waveform parameters.  It holds none of the method's arithmetic (no
finite-element matrices, no time stepping, no Parareal) and is the one module
shared by the CPU oracle and the GPU path.

The paper's example (Section 4) is a nonlinear 2-D coaxial cable driven by a
50 Hz sinusoidal current over one period T = 0.02 s; its geometry and B-H data
come from a reference that is not reproduced in the paper.  The workloads here
stand in for it with a structured polar P1 triangulation:

* node 0 is the centre; node ``1 + (i-1)*ntheta + j`` sits at radius ``r_i``,
  angle ``2*pi*j/ntheta`` for rings i = 1..nr, j = 0..ntheta-1;
* the centre fan is ``(0, (1,j), (1,j+1))``; each quad between rings i and i+1
  is split into ``((i,j),(i+1,j),(i+1,j+1))`` and ``((i,j),(i+1,j+1),(i,j+1))``;
* ring radii are piecewise uniform and conform to every material interface;
  rings are shared between layers in proportion to thickness, rounded by the
  largest-remainder rule;
* the outer ring carries the homogeneous Dirichlet condition A = 0.

Reluctivity models (per material): model 0 is linear with a constant ``nu``;
model 1 is the Brauer law ``nu(b2) = k1*exp(k2*b2) + k3`` with ``b2 = |B|^2``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MU0 = 4.0e-7 * math.pi
NU0 = 1.0 / MU0
SIGMA_CU = 5.8e7

# material models
LINEAR = 0
BRAUER = 1


@dataclass
class Layer:
    r_out: float          # outer radius of the layer (m)
    sigma: float          # conductivity (S/m)
    mat: int              # index into the material table
    drive: int = 0        # +1 / -1: carries +i(t) / -i(t) spread uniformly; 0: none


@dataclass
class Problem:
    """Everything a solver needs, as plain arrays (0-based indices)."""
    name: str
    xy: np.ndarray            # float64 [n_nodes, 2]
    tri: np.ndarray           # int32   [n_tri, 3]
    dirichlet: np.ndarray     # int32   [n_dir], A = 0 there
    sigma: np.ndarray         # float64 [n_tri]
    mat_id: np.ndarray        # int32   [n_tri]
    mat_model: np.ndarray     # int32   [n_mat] (LINEAR / BRAUER)
    mat_par: np.ndarray       # float64 [n_mat, 4] = (nu, k1, k2, k3)
    js: np.ndarray            # float64 [n_tri] source density per ampere (A/m^2 per A)
    f0: float                 # fundamental frequency (Hz)
    orders: np.ndarray        # int32   [n_h] harmonic orders of i(t)
    amps: np.ndarray          # float64 [n_h] amplitudes (A)
    phases: np.ndarray        # float64 [n_h] phases (rad)
    T: float                  # period (s)
    N: int                    # Parareal subintervals
    m: int                    # fine implicit-Euler steps per subinterval
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])

    def current(self, t):
        """Imposed current i(t) = sum_h amp_h sin(2*pi*order_h*f0*t + phase_h)."""
        t = np.asarray(t, dtype=np.float64)
        out = np.zeros_like(t)
        for o, a, p in zip(self.orders, self.amps, self.phases):
            out = out + a * np.sin(2.0 * math.pi * float(o) * self.f0 * t + p)
        return out


def ring_counts(thicknesses, nr):
    """Share nr rings between layers in proportion to thickness (largest remainder)."""
    th = np.asarray(thicknesses, dtype=np.float64)
    quota = nr * th / th.sum()
    base = np.floor(quota).astype(int)
    rem = nr - int(base.sum())
    order = np.argsort(-(quota - base), kind="stable")
    base[order[:rem]] += 1
    if np.any(base < 1):
        raise ValueError("nr too small to give every layer a ring")
    return base


def ring_radii(interfaces, counts):
    """Piecewise-uniform ring radii r_1..r_nr; interfaces[k] is layer k's outer radius."""
    radii = []
    r0 = 0.0
    for r1, c in zip(interfaces, counts):
        radii.extend(r0 + (r1 - r0) * np.arange(1, c + 1) / c)
        r0 = r1
    return np.asarray(radii, dtype=np.float64)


def polar_mesh(radii, ntheta):
    """Centre node + rings; returns xy, tri (int32, counter-clockwise), dirichlet ring,
    and for each triangle the ring index of its outer edge (1..nr)."""
    nr = len(radii)
    theta = 2.0 * math.pi * np.arange(ntheta) / ntheta
    xy = np.zeros((1 + nr * ntheta, 2), dtype=np.float64)
    for i, r in enumerate(radii):
        xy[1 + i * ntheta: 1 + (i + 1) * ntheta, 0] = r * np.cos(theta)
        xy[1 + i * ntheta: 1 + (i + 1) * ntheta, 1] = r * np.sin(theta)

    def node(i, j):  # ring i in 1..nr
        return 1 + (i - 1) * ntheta + (j % ntheta)

    tris = []
    ring_of = []
    for j in range(ntheta):
        tris.append((0, node(1, j), node(1, j + 1)))
        ring_of.append(1)
    for i in range(1, nr):
        for j in range(ntheta):
            tris.append((node(i, j), node(i + 1, j), node(i + 1, j + 1)))
            tris.append((node(i, j), node(i + 1, j + 1), node(i, j + 1)))
            ring_of.extend((i + 1, i + 1))
    tri = np.asarray(tris, dtype=np.int32)
    dirichlet = np.arange(1 + (nr - 1) * ntheta, 1 + nr * ntheta, dtype=np.int32)
    return xy, tri, dirichlet, np.asarray(ring_of, dtype=np.int32)


def polygon_ring_area(r_in, r_out, ntheta):
    """Area between two inscribed regular ntheta-gons (exact for the polar mesh)."""
    return 0.5 * ntheta * math.sin(2.0 * math.pi / ntheta) * (r_out ** 2 - r_in ** 2)


def layered_coax(name, layers, materials, nr, ntheta, f0, orders, amps, phases,
                 T, N, m, meta=None):
    interfaces = [L.r_out for L in layers]
    thick = np.diff(np.concatenate([[0.0], interfaces]))
    counts = ring_counts(thick, nr)
    radii = ring_radii(interfaces, counts)
    xy, tri, dirichlet, ring_of = polar_mesh(radii, ntheta)
    # layer of each ring: ring index (1-based) -> layer k
    ring_layer = np.repeat(np.arange(len(layers)), counts)     # for rings 1..nr
    tri_layer = ring_layer[ring_of - 1]
    sigma = np.array([layers[k].sigma for k in tri_layer], dtype=np.float64)
    mat_id = np.array([layers[k].mat for k in tri_layer], dtype=np.int32)
    js = np.zeros(len(tri), dtype=np.float64)
    r_in = 0.0
    for k, L in enumerate(layers):
        if L.drive != 0:
            js[tri_layer == k] = L.drive / polygon_ring_area(r_in, L.r_out, ntheta)
        r_in = L.r_out
    mat_model = np.array([mm[0] for mm in materials], dtype=np.int32)
    mat_par = np.array([mm[1:] for mm in materials], dtype=np.float64).reshape(-1, 4)
    info = dict(nr=nr, ntheta=ntheta, ring_counts=counts.tolist(),
                interfaces=list(interfaces))
    if meta:
        info.update(meta)
    return Problem(name=name, xy=xy, tri=tri, dirichlet=dirichlet, sigma=sigma,
                   mat_id=mat_id, mat_model=mat_model, mat_par=mat_par, js=js,
                   f0=float(f0), orders=np.asarray(orders, dtype=np.int32),
                   amps=np.asarray(amps, dtype=np.float64),
                   phases=np.asarray(phases, dtype=np.float64),
                   T=float(T), N=int(N), m=int(m), meta=info)


AIR = (LINEAR, NU0, 0.0, 0.0, 0.0)


def steel(k1=3.8, k2=2.17, k3=396.2):
    return (BRAUER, 0.0, k1, k2, k3)


def c1(nr=20, ntheta=40, N=10, m=20):
    """Linear coax: copper core, insulation, copper return conductor, air; 1 A at 50 Hz.
    The return current flows in the outer conductor."""
    layers = [Layer(1e-3, SIGMA_CU, 0, +1), Layer(2e-3, 0.0, 0),
              Layer(2.5e-3, SIGMA_CU, 0, -1), Layer(3e-3, 0.0, 0)]
    return layered_coax("C1-linear", layers, [AIR], nr, ntheta, 50.0, [1], [1.0], [0.0],
                        0.02, N, m)


def c2(nr=60, ntheta=120, N=40, m=50, seed=2, sheath_sigma=2e6):
    """Nonlinear coax: the air layer of C1 becomes a Brauer steel sheath.  The core alone
    is driven (the return closes at the outer boundary) so that the sheath saturates;
    amplitude 200 + 600*U with U from the seed."""
    amp = 200.0 + 600.0 * np.random.default_rng(seed).random()
    layers = [Layer(1e-3, SIGMA_CU, 0, +1), Layer(2e-3, 0.0, 0),
              Layer(2.5e-3, SIGMA_CU, 0), Layer(3e-3, sheath_sigma, 1)]
    return layered_coax("C2-nonlinear", layers, [AIR, steel()], nr, ntheta, 50.0, [1],
                        [amp], [0.0], 0.02, N, m, meta=dict(seed=seed))


def c2lin(nr=60, ntheta=120, N=40, m=50, seed=2, f_scale=1.0):
    """C2 with the sheath's Brauer law replaced by a linear material at the steel's
    unsaturated reluctivity nu(0) = k1 + k3; frequency and period scaled by f_scale
    (f0 = 50 f_scale Hz, T = 0.02 / f_scale).  The sheath's magnetic time constant then
    sets how many periods classical time stepping needs, without saturation."""
    amp = 200.0 + 600.0 * np.random.default_rng(seed).random()
    k1, _, k3 = 3.8, 2.17, 396.2
    layers = [Layer(1e-3, SIGMA_CU, 0, +1), Layer(2e-3, 0.0, 0),
              Layer(2.5e-3, SIGMA_CU, 0), Layer(3e-3, 2e6, 1)]
    return layered_coax("C2-linearised", layers, [AIR, (LINEAR, k1 + k3, 0.0, 0.0, 0.0)], nr, ntheta,
                        50.0 * f_scale, [1], [amp], [0.0], 0.02 / f_scale, N, m,
                        meta=dict(seed=seed, f_scale=f_scale))


def c3(nr=400, ntheta=800, N=200, m=100, seed=3):
    """Large nonlinear coax: fundamental plus a 20% third harmonic with a seeded phase."""
    rng = np.random.default_rng(seed)
    amp = 200.0 + 600.0 * rng.random()
    phi3 = 2.0 * math.pi * rng.random()
    layers = [Layer(1e-3, SIGMA_CU, 0, +1), Layer(2e-3, 0.0, 0),
              Layer(2.5e-3, SIGMA_CU, 0), Layer(3e-3, 2e6, 1)]
    return layered_coax("C3-large", layers, [AIR, steel()], nr, ntheta, 50.0, [1, 3],
                        [amp, 0.2 * amp], [0.0, phi3], 0.02, N, m, meta=dict(seed=seed))


def c4_designs(n_designs=256, seed=4, N=40, m=50):
    """Batch of nonlinear coax designs of uneven size; draw order per design:
    nr, sheath thickness, sheath conductivity (log-uniform), Brauer k2, amplitude."""
    rng = np.random.default_rng(seed)
    out = []
    for d in range(n_designs):
        nr = int(rng.integers(20, 201))
        t = float(rng.uniform(0.2e-3, 1.0e-3))
        sig = float(10.0 ** rng.uniform(5.0, 7.0))
        k2 = float(rng.uniform(1.5, 3.0))
        amp = float(rng.uniform(100.0, 800.0))
        layers = [Layer(1e-3, SIGMA_CU, 0, +1), Layer(2e-3, 0.0, 0),
                  Layer(2.5e-3, SIGMA_CU, 0), Layer(2.5e-3 + t, sig, 1)]
        out.append(layered_coax(f"C4-design{d}", layers, [AIR, steel(k2=k2)], nr, 2 * nr,
                                50.0, [1], [amp], [0.0], 0.02, N, m,
                                meta=dict(seed=seed, design=d, sheath=t)))
    return out


def c5_small(seed=5):
    """Adjoint case (i): the C1 mesh with C2's materials (steel sheath, core-only drive)."""
    amp = 200.0 + 600.0 * np.random.default_rng(seed).random()
    layers = [Layer(1e-3, SIGMA_CU, 0, +1), Layer(2e-3, 0.0, 0),
              Layer(2.5e-3, SIGMA_CU, 0), Layer(3e-3, 2e6, 1)]
    return layered_coax("C5-small", layers, [AIR, steel()], 20, 40, 50.0, [1], [amp],
                        [0.0], 0.02, 10, 20, meta=dict(seed=seed))


def tiny(nr=4, ntheta=8, N=4, m=3, nonlinear=False, amp=None, sheath_sigma=2e6,
         f_scale=1.0):
    """Small variants of C1/C2 for brute-force and property tests."""
    if nonlinear:
        a = 400.0 if amp is None else amp
        layers = [Layer(1e-3, SIGMA_CU, 0, +1), Layer(2e-3, 0.0, 0),
                  Layer(2.5e-3, SIGMA_CU, 0), Layer(3e-3, sheath_sigma, 1)]
        mats = [AIR, steel()]
    else:
        a = 1.0 if amp is None else amp
        layers = [Layer(1e-3, SIGMA_CU, 0, +1), Layer(2e-3, 0.0, 0),
                  Layer(2.5e-3, SIGMA_CU, 0, -1), Layer(3e-3, 0.0, 0)]
        mats = [AIR]
    return layered_coax(f"tiny-{'nl' if nonlinear else 'lin'}-{nr}x{ntheta}", layers, mats,
                        nr, ntheta, 50.0 * f_scale, [1], [a], [0.0], 0.02 / f_scale, N, m)


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c5": c5_small}


def chain_starts(prob, free, seed, amp=1e-4):
    """Seeded chain starts for fine-sweep parity cases, rows n = 0..N-1 over the free nodes
    `free`: a radial profile amp (R - r)/R, R the outer radius, scaled per row by
    1 + 0.1 g_n with g_n standard normal from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    r = np.hypot(prob.xy[free, 0], prob.xy[free, 1])
    R = float(np.hypot(prob.xy[:, 0], prob.xy[:, 1]).max())
    return np.outer(1.0 + 0.1 * rng.standard_normal(prob.N), amp * (R - r) / R)


def random_rows(N, n, seed, amp):
    """Seeded samples for coarse-correction parity cases: amp times standard normal
    values from default_rng(seed), shape [N, n]."""
    return amp * np.random.default_rng(seed).standard_normal((N, n))


def sample_index(n, count, seed):
    """Sorted distinct indices into 0..n-1 at which large parity cases compare values:
    index 0 (the centre node's row) plus count - 1 drawn by default_rng(seed)."""
    rng = np.random.default_rng(seed)
    pick = rng.choice(np.arange(1, n), size=min(count, n) - 1, replace=False)
    return np.sort(np.concatenate([[0], pick])).astype(np.int64)
