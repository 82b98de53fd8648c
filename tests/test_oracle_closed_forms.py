"""Pins of the oracle against closed forms of the axisymmetric coax (Section 4 model class):

* static field of a DC current (Ampere's law, piecewise r^2 / ln r);
* linear eddy currents in the frequency domain (modified Bessel functions per layer);
* saturated static field in the Brauer sheath (scalar root of nu(B^2) B = H per radius).

Each check also demands second-order convergence of the RMS nodal error under mesh
refinement, so a wrong
factor anywhere in K, M, F or the reluctivity shows up as an O(1) error."""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.optimize as so
import scipy.sparse.linalg as spla
import scipy.special as ss

from oracle.fe import FE
from oracle.timestep import ie_step
from workloads import coax

A_, B_, C_, R_ = 1e-3, 2e-3, 2.5e-3, 3e-3


def _rms(e):
    """RMS nodal error (the max-norm is dominated by the centre node of the fan)."""
    return float(np.sqrt(np.mean(np.abs(e) ** 2)))


def _radius(fe):
    return np.hypot(fe.prob.xy[fe.free, 0], fe.prob.xy[fe.free, 1])


def _dc_closed_form(r, I):
    """A(r) = mu0/(2 pi) int_r^R I_enc(s)/s ds with core +I and outer conductor -I."""
    k = coax.MU0 / (2 * math.pi)
    G_b = I / (C_ ** 2 - B_ ** 2) * (C_ ** 2 * math.log(C_ / B_) - (C_ ** 2 - B_ ** 2) / 2)
    out = np.zeros_like(r)
    m = r < A_
    out[m] = I * (A_ ** 2 - r[m] ** 2) / (2 * A_ ** 2) + I * math.log(B_ / A_) + G_b
    m = (r >= A_) & (r < B_)
    out[m] = I * np.log(B_ / r[m]) + G_b
    m = (r >= B_) & (r < C_)
    out[m] = I / (C_ ** 2 - B_ ** 2) * (C_ ** 2 * np.log(C_ / r[m]) - (C_ ** 2 - r[m] ** 2) / 2)
    return k * out


def test_static_dc_field_second_order():
    errs = []
    for nr in (12, 24, 48):
        fe = FE(coax.c1(nr=nr, ntheta=2 * nr))
        K = fe.K_matrix(np.full(fe.prob.n_tri, coax.NU0))
        u = spla.spsolve(K.tocsc(), 1.0 * fe.F)
        ex = _dc_closed_form(_radius(fe), 1.0)
        errs.append(_rms(u - ex) / np.abs(ex).max())
    assert errs[-1] < 2e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def _skin_closed_form(r, omega, I):
    """Phasor A(r) of -nu0 A'' - nu0 A'/r + i omega sigma A = Js per layer (C1 layout),
    A regular at 0, A and A' continuous, A(R) = 0."""
    nu, sig = coax.NU0, coax.SIGMA_CU
    k = np.sqrt(1j * omega * sig / nu)
    Jc = I / (math.pi * A_ ** 2)
    Jo = -I / (math.pi * (C_ ** 2 - B_ ** 2))
    pc, po = Jc / (1j * omega * sig), Jo / (1j * omega * sig)
    I0, I1, K0, K1 = (lambda x: ss.iv(0, x)), (lambda x: ss.iv(1, x)), (lambda x: ss.kv(0, x)), (lambda x: ss.kv(1, x))
    # unknowns: c1 (core I0), d1, d2 (ins: d1 + d2 ln r), e1, e2 (outer I0, K0), g1, g2 (air)
    M = np.zeros((7, 7), complex)
    rhs = np.zeros(7, complex)
    # r = a: core = ins
    M[0, 0] = I0(k * A_); M[0, 1] = -1; M[0, 2] = -math.log(A_); rhs[0] = -pc
    M[1, 0] = k * I1(k * A_); M[1, 2] = -1 / A_
    # r = b: ins = outer
    M[2, 1] = 1; M[2, 2] = math.log(B_); M[2, 3] = -I0(k * B_); M[2, 4] = -K0(k * B_); rhs[2] = po
    M[3, 2] = 1 / B_; M[3, 3] = -k * I1(k * B_); M[3, 4] = k * K1(k * B_)
    # r = c: outer = air
    M[4, 3] = I0(k * C_); M[4, 4] = K0(k * C_); M[4, 5] = -1; M[4, 6] = -math.log(C_); rhs[4] = -po
    M[5, 3] = k * I1(k * C_); M[5, 4] = -k * K1(k * C_); M[5, 6] = -1 / C_
    # r = R: A = 0
    M[6, 5] = 1; M[6, 6] = math.log(R_)
    c = np.linalg.solve(M, rhs)
    out = np.zeros(r.shape, complex)
    m = r < A_
    out[m] = pc + c[0] * I0(k * r[m])
    m = (r >= A_) & (r < B_)
    out[m] = c[1] + c[2] * np.log(r[m])
    m = (r >= B_) & (r < C_)
    out[m] = po + c[3] * I0(k * r[m]) + c[4] * K0(k * r[m])
    m = r >= C_
    out[m] = c[5] + c[6] * np.log(r[m])
    return out


@pytest.mark.parametrize("freq", [50.0, 4.37e3])
def test_linear_skin_effect_bessel(freq):
    """(K + i omega M) A = F against the Bessel solution; 4.37 kHz puts one skin depth
    across the copper core, so the conductivity mass matters at O(1)."""
    omega = 2 * math.pi * freq
    errs = []
    for nr in (12, 24, 48):
        fe = FE(coax.c1(nr=nr, ntheta=2 * nr))
        K = fe.K_matrix(np.full(fe.prob.n_tri, coax.NU0))
        A = (K + 1j * omega * fe.M).astype(complex).tocsc()
        u = spla.spsolve(A, fe.F.astype(complex))
        ex = _skin_closed_form(_radius(fe), omega, 1.0)
        errs.append(_rms(u - ex) / np.abs(ex).max())
    assert errs[-1] < 3e-3, errs
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs
    if freq > 1e3:
        # the eddy-current part is far from negligible at this frequency
        fe = FE(coax.c1(nr=40, ntheta=80))
        K = fe.K_matrix(np.full(fe.prob.n_tri, coax.NU0))
        static = spla.spsolve(K.tocsc(), fe.F)
        ex = _skin_closed_form(_radius(fe), omega, 1.0)
        assert np.abs(ex - static).max() > 0.1 * np.abs(ex).max()


def _static_sheath_closed_form(r, I, k1=3.8, k2=2.17, k3=396.2):
    """Core-only DC current I; H = I_enc/(2 pi r); in the Brauer sheath nu(B^2) B = H."""
    mu0 = coax.MU0

    def B(s):
        Ienc = I * min(1.0, (s / A_) ** 2)
        H = Ienc / (2 * math.pi * s) if s > 0 else 0.0
        if s >= C_:
            return so.brentq(lambda b: (k1 * math.exp(k2 * b * b) + k3) * b - H, 0.0, 10.0, xtol=1e-15)
        return mu0 * H

    out = np.zeros_like(r)
    for i, ri in enumerate(r):
        lo = max(ri, 0.0)
        pieces = [p for p in (A_, B_, C_) if p > lo] + [R_]
        acc, a = 0.0, lo
        for b in pieces:
            acc += si.quad(B, a, b, epsabs=1e-16, epsrel=1e-12, limit=200)[0]
            a = b
        out[i] = acc
    return out


def test_static_saturated_sheath_second_order():
    I = 500.0
    errs = []
    for nr in (12, 24, 48):
        prob = coax.c2(nr=nr, ntheta=2 * nr)
        prob.f0 = 0.0                              # i(t) = I sin(pi/2) = I: a DC current
        prob.amps = np.array([I])
        prob.phases = np.array([math.pi / 2])
        fe = FE(prob)
        u, _ = ie_step(fe, np.zeros(fe.n), 0.0, 1e30)   # M/dt -> 0: K(u) u = I F
        r = _radius(fe)
        ex = _static_sheath_closed_form(r, I)
        errs.append(_rms(u - ex) / np.abs(ex).max())
        _, _, b2, _, _ = fe.element_state(u)
    assert math.sqrt(b2.max()) > 1.8                   # the sheath is saturated
    assert errs[-1] < 5e-3, errs
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs
