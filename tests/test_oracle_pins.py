"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks the oracle against something fixed by the physics, the
mathematics or an independent published value: textbook cross sections,
four-vector kinematics, closed forms, exact polynomial structure, symmetry,
finite differences, brute force on tiny inputs.  A dropped term, a wrong sign,
index or transposed operand anywhere in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "textbook.json")))
HBARC2 = GOLD["hbarc2_MeV2_cm2"]["value"]

# Constants of the reading (the oracle keeps its own copy; these are the
# test's, used only to build kinematics and closed forms).
ME, GF, SW2 = 0.51099895, 1.1663788e-11, 0.23122
SM = oracle.THETA_SM


def th(**kw):
    t = SM.copy()
    names = ["eLL", "eRR", "tLL", "tRR", "m2", "f8", "fb"]
    for k, v in kw.items():
        t[names.index(k)] = v
    return t


@pytest.fixture(scope="module")
def bare():
    """An oracle with no sources: only the cross-section entry is used."""
    return oracle.Oracle()


# ---------------------------------------------------------------- kinematics
def recoil_tmax(E):
    """Forward electron (theta_e = 0) recoil energy from the textbook angle
    relation T = 2 m E^2 cos^2 / ((m+E)^2 - E^2 cos^2)."""
    c2 = 1.0
    return 2 * ME * E * E * c2 / ((ME + E) ** 2 - E * E * c2)


def four_vectors(E, T):
    """Lab-frame four-momenta for nu(E) e(rest) -> nu' e'(T)."""
    pe = math.sqrt(T * T + 2 * ME * T)
    cos_e = (E + ME) / E * math.sqrt(T / (T + 2 * ME))
    sin_e = math.sqrt(max(0.0, 1 - cos_e * cos_e))
    k = np.array([E, 0, 0, E])
    p = np.array([ME, 0, 0, 0])
    pp = np.array([ME + T, pe * sin_e, 0, pe * cos_e])
    kp = k + p - pp
    return k, p, kp, pp


def dot(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


@pytest.mark.parametrize("E,printed", [(0.42, 0.261140), (0.862, 0.664917),
                                       (1.44, 1.223002), (1.73, 1.507379),
                                       (16.0, 15.748516)])
def test_compton_edge_of_lines(E, printed):
    """A single line: the oracle's spectrum is non-zero exactly in the bins
    whose centre lies below the forward-recoil energy."""
    assert recoil_tmax(E) == pytest.approx(printed, abs=2e-6)
    o = oracle.Oracle()
    n_t = 16000
    o.set_sources([dict(kind=0, E=[E], weight=[1.0], p_ee=[0.55], group=0)],
                  n_t)
    S = o.spectrum(SM)
    centres = (np.arange(n_t) + 0.5) * 16.0 / n_t
    tm = recoil_tmax(E)
    assert np.all(S[centres <= tm] > 0)
    assert np.all(S[centres > tm] == 0)
    # the kinematic outgoing state really is on shell at T_max
    k, p, kp, pp = four_vectors(E, tm * (1 - 1e-12))
    assert abs(dot(kp, kp)) < 1e-9 * E * E


def test_matrix_element_route(bare):
    """dsigma/dT against the chiral-coupling squared amplitude built from
    explicit four-vectors: 2 G_F^2/(pi m E^2) * [gL^2 (k.p)(k'.p') +
    gR^2 (k.p')(k'.p) - gL gR m^2 (k.k')] (neutral + charged current with
    V-A neutrinos; e.g. Giunti & Kim, Fundamentals of Neutrino Physics)."""
    g = synth.rng(7)
    for _ in range(200):
        E = g.uniform(0.1, 20.0)
        T = g.uniform(1e-4, 0.999) * recoil_tmax(E)
        t = th(eLL=g.uniform(-.5, .5), eRR=g.uniform(-.5, .5),
               tLL=g.uniform(-.5, .5), tRR=g.uniform(-.5, .5))
        k, p, kp, pp = four_vectors(E, T)
        for a, (gl, gr) in enumerate([(0.5 + SW2 + t[0], SW2 + t[1]),
                                      (-0.5 + SW2, SW2),
                                      (-0.5 + SW2 + t[2], SW2 + t[3])]):
            F = (gl * gl * dot(k, p) * dot(kp, pp) + gr * gr * dot(k, pp)
                 * dot(kp, p) - gl * gr * ME * ME * dot(k, kp))
            ref = 2 * GF * GF / (math.pi * ME * E * E) * F
            got = bare.dsigma(a, E, T, t)
            assert got == pytest.approx(ref, rel=1e-9, abs=1e-12 * abs(ref)
                                        + 1e-40)


def test_magnetic_moment_prefactor(bare):
    """(pi alpha^2/m_e^2) = 2.495e-25 cm^2 per (mu_nu/mu_B)^2 per (1/T-1/E)."""
    E, T = 10.0, 1.0
    d1 = bare.dsigma(0, E, T, th(m2=1.0))
    d0 = bare.dsigma(0, E, T, SM)
    mm = (d1 - d0) / (1e-22 * (1 / T - 1 / E)) * HBARC2
    assert mm == pytest.approx(GOLD["mm_prefactor_cm2"]["value"],
                               rel=GOLD["mm_prefactor_cm2"]["rel_tol"])
    # incoherent sum: the magnetic term is the same for every flavour
    for a in (1, 2):
        da = bare.dsigma(a, E, T, th(m2=1.0)) - bare.dsigma(a, E, T, SM)
        assert da == pytest.approx(d1 - d0, rel=1e-12)


@pytest.mark.parametrize("flavour,key", [(0, "sigma_nue_e_per_GeV_cm2"),
                                         (1, "sigma_numu_e_per_GeV_cm2"),
                                         (2, "sigma_numu_e_per_GeV_cm2")])
def test_high_energy_total_cross_section(bare, flavour, key):
    """Integral of dsigma/dT over the kinematic range at E = 200 MeV, per
    GeV, against the textbook tree-level value."""
    E = 200.0
    f = lambda T: bare.dsigma(flavour, E, T, SM)
    sig, _ = integrate.quad(f, 0.0, recoil_tmax(E), limit=200, epsrel=1e-10)
    per_gev = sig * HBARC2 / (E / 1000.0)
    assert per_gev == pytest.approx(GOLD[key]["value"],
                                    rel=GOLD[key]["rel_tol"])


@pytest.mark.parametrize("flavour,printed", [(0, 5.945e-45), (1, 1.252e-45)])
def test_line_total_cross_section_closed_form(bare, flavour, printed):
    """Closed-form integral of the weak cross section at the 7Be energy."""
    E = 0.862
    tm = recoil_tmax(E)
    gl = (0.5 if flavour == 0 else -0.5) + SW2
    gr = SW2
    pref = 2 * GF * GF * ME / math.pi
    closed = pref * (gl * gl * tm + gr * gr * E / 3 * (1 - (1 - tm / E) ** 3)
                     - gl * gr * ME * tm * tm / (2 * E * E))
    sig, _ = integrate.quad(lambda T: bare.dsigma(flavour, E, T, SM), 0, tm,
                            epsrel=1e-12)
    assert sig == pytest.approx(closed, rel=1e-10)
    assert closed * HBARC2 == pytest.approx(printed, rel=2e-3)


def test_helicity_limits(bare):
    """Pure left-handed electron coupling gives a flat recoil spectrum, pure
    right-handed gives (1 - T/E)^2 (helicity structure of the amplitude)."""
    E = 5.0
    Ts = np.linspace(0.01, recoil_tmax(E) * 0.999, 13)
    flat = [bare.dsigma(0, E, T, th(eRR=-SW2)) for T in Ts]
    assert np.ptp(flat) <= 1e-13 * abs(flat[0])
    right = np.array([bare.dsigma(0, E, T, th(eLL=-0.5 - SW2)) for T in Ts])
    shape = right / (1 - Ts / E) ** 2
    assert np.ptp(shape) <= 1e-12 * abs(shape[0])


def test_e_integral_matches_quadrature():
    """Eq. (fT) with many midpoint nodes converges to the continuous
    integral over E from the kinematic minimum up to the endpoint."""
    e0, flux = 1.73, 1.0
    n_e = 8192
    src = synth.source_nodes(n_e, sources=(("CNO", "beta", e0, flux, 0),))
    o = oracle.Oracle()
    n_t = 40
    o.set_sources(src, n_t, 0.0, 1.6)
    t = th(eLL=0.2, eRR=-0.3, tLL=0.1, tRR=0.25, m2=4.0)
    S = o.spectrum(t)
    bare = oracle.Oracle()

    def integrand(E, T):
        pe = synth.survival_prob(E)
        P = [pe, (1 - pe) / 2, (1 - pe) / 2]
        return synth.beta_shape(E, e0) * sum(
            P[a] * bare.dsigma(a, E, T, t) for a in range(3))

    for l in (0, 7, 19, 31, 36):
        T = (l + 0.5) * 1.6 / n_t
        emin = (T + math.sqrt(T * T + 2 * ME * T)) / 2
        ref, _ = integrate.quad(integrand, emin, e0, args=(T,), epsrel=1e-11)
        # midpoint rule with a jump at E_min: O(dE) error
        assert S[l] == pytest.approx(ref, rel=3e-3 * (e0 / n_e) / 2e-4)


# --------------------------------------------------------- small analysis
@pytest.fixture(scope="module")
def small():
    """Config-0-like analysis with a reduced MC sample."""
    src = synth.source_nodes(64)
    rsp = synth.response_mc(96, 48, 200_000, seed=11)
    o = oracle.Oracle()
    o.set_sources(src, 96)
    o.set_response(rsp.R, n_sig=1e4)
    mu_sm = o.mu(SM)
    b = np.full(48, 10.0)
    o.set_data(synth.poisson_data(mu_sm + b, 5), b)
    return o, rsp, b


def test_sm_limit_exact(small):
    """At the SM point the weights are exactly one (the paper: the SM
    prediction is recovered by construction) and mu is the plain fold."""
    o, rsp, b = small
    w = o.weights(SM)
    assert np.all(w == 1.0)
    m = o.row_factors()
    ref = b + (m[:, None] * rsp.R.astype(np.float64)).sum(0)
    assert np.allclose(o.mu(SM), ref, rtol=1e-13, atol=0)


def test_row_factors_are_normalised_sm_reference(small):
    o, rsp, b = small
    m = o.row_factors()
    S = o.spectrum(SM)
    assert m.sum() == pytest.approx(1e4, rel=1e-13)
    nz = S > 0
    assert np.allclose(m[nz] / S[nz], 1e4 / S.sum(), rtol=1e-13)
    assert np.all(m[~nz] == 0)


def test_response_conservation():
    rsp = synth.response_mc(64, 40, 300_000, seed=3)
    assert rsp.row_events.sum() == 300_000
    assert np.array_equal(rsp.counts.sum(1) + rsp.under + rsp.over,
                          rsp.row_events)
    eff = rsp.R.astype(np.float64).sum(1)
    assert np.all(eff <= 1 + 1e-6)
    assert np.allclose(eff, 1 - (rsp.under + rsp.over) / rsp.row_events,
                       atol=1e-6)
    again = synth.response_mc(64, 40, 300_000, seed=3)
    assert np.array_equal(again.counts, rsp.counts)


def test_nll_brute_force():
    """Eq. (logL) on a 4x3 hand-made problem, summed term by term with
    math.lgamma, including n = 0 and non-integer (Asimov) counts."""
    o = oracle.Oracle()
    o.set_sources([dict(kind=0, E=[0.862], weight=[1.0], p_ee=[0.5],
                        group=0)], 4, 0.0, 0.8)
    R = np.array([[0.5, 0.25, 0.125], [0.0, 0.75, 0.25], [0.25, 0.25, 0.5],
                  [1.0, 0.0, 0.0]], dtype=np.float32)
    m = np.array([3.0, 5.0, 7.0, 11.0])
    o.set_response(R, m=m)
    n = np.array([0.0, 7.0, 3.5])
    b = np.array([1.0, 2.0, 0.5])
    o.set_data(n, b)
    # SM point: w = 1 in every non-empty bin (bin 3 lies above the edge
    # and gets w = 1 by definition)
    mu = [sum(m[l] * float(R[l, j]) for l in range(4)) + b[j]
          for j in range(3)]
    ref = 2 * sum(mu[j] - (n[j] * math.log(mu[j]) if n[j] else 0)
                  + math.lgamma(n[j] + 1) for j in range(3))
    assert o.nll(SM) == pytest.approx(ref, rel=1e-14)
    # f_bkg scales b only
    t = th(fb=0.25)
    mu2 = [mu[j] - 0.75 * b[j] for j in range(3)]
    ref2 = 2 * sum(mu2[j] - (n[j] * math.log(mu2[j]) if n[j] else 0)
                   + math.lgamma(n[j] + 1) for j in range(3))
    assert o.nll(t) == pytest.approx(ref2, rel=1e-14)
    # pulls
    o.set_data(n, b, pull_mean=[0, 0, 0, 0, 0, 1, 1],
               pull_sigma=[0, 0, 0, 0, 0, 0.1, 0.2])
    assert o.nll(t) == pytest.approx(ref2 + (0.75 / 0.2) ** 2, rel=1e-14)
    # a non-positive expectation under data is impossible: +inf
    o.set_data(n, b)
    R0 = R.copy()
    R0[:, 1] = 0
    o.set_response(R0, m=m)
    assert o.nll(th(fb=-1.0)) == math.inf


def test_gradient_with_empty_bin():
    """Eq. (logL) at a bin with n_j = 0 is the term 2 mu_j, whose derivative
    is 2 also where mu_j = 0 (an empty response column with no background):
    the analytic gradient stays finite there and equals central differences
    of -2lnL, on the 4x3 problem above widened by such a column."""
    o = oracle.Oracle()
    o.set_sources([dict(kind=0, E=[0.862], weight=[1.0], p_ee=[0.5],
                        group=0),
                   dict(kind=0, E=[1.44], weight=[0.3], p_ee=[0.45],
                        group=1)], 4, 0.0, 1.6)
    R = np.array([[0.5, 0.25, 0.125, 0.0], [0.0, 0.75, 0.25, 0.0],
                  [0.25, 0.25, 0.5, 0.0], [1.0, 0.0, 0.0, 0.0]],
                 dtype=np.float32)
    m = np.array([3.0, 5.0, 7.0, 11.0])
    o.set_response(R, m=m)
    n = np.array([0.0, 7.0, 3.5, 0.0])
    b = np.array([1.0, 2.0, 0.5, 0.0])
    o.set_data(n, b, pull_mean=[0, 0, 0, 0, 0, 1, 1],
               pull_sigma=[0, 0, 0, 0, 0, 0.1, 0.2])
    t = th(eLL=0.1, eRR=-0.2, tLL=0.3, tRR=0.05, m2=3.0, f8=1.1, fb=0.9)
    assert o.mu(t)[3] == 0.0
    v, g = o.nll_grad(t)
    assert np.all(np.isfinite(g)) and v == pytest.approx(o.nll(t), rel=1e-14)
    h = 1e-3
    for i in range(7):
        def f(s):
            tt = t.copy()
            tt[i] += s * h
            return o.nll(tt)
        fd = (8 * (f(1) - f(-1)) - (f(2) - f(-2))) / (12 * h)
        assert g[i] == pytest.approx(fd, rel=1e-8, abs=1e-9), i
    # the empty bin's term is 2 mu_3 = 0 whatever theta is, so f_bkg's
    # derivative is the sum over the other bins of 2 (1 - n_j/mu_j) b_j plus
    # the pull, written out by hand
    mu = o.mu(t)
    ref = sum((2.0 if n[j] == 0 else 2 * (1 - n[j] / mu[j])) * b[j]
              for j in range(3)) + 2 * (t[6] - 1) / 0.2 ** 2
    assert g[6] == pytest.approx(ref, rel=1e-13)


def test_polynomial_structure(small):
    """S_theta is exactly quadratic in each eps, linear in m2 and f_8B;
    mu is linear in f_bkg."""
    o, rsp, b = small
    base = th(eLL=0.1, eRR=-0.2, tLL=0.3, tRR=0.05, m2=3.0, f8=1.1, fb=0.9)
    S0 = o.spectrum(base)
    sc = np.abs(S0).max()
    for i in range(4):
        vals = []
        for s in range(4):
            t = base.copy()
            t[i] += 0.37 * s
            vals.append(o.spectrum(t))
        third = vals[3] - 3 * vals[2] + 3 * vals[1] - vals[0]
        assert np.abs(third).max() <= 1e-12 * sc
        second = vals[2] - 2 * vals[1] + vals[0]
        assert np.abs(second).max() > 1e-6 * sc
    for i in (4, 5):
        t1, t2 = base.copy(), base.copy()
        t1[i] += 1.3
        t2[i] += 2.6
        d2 = o.spectrum(t2) - 2 * o.spectrum(t1) + S0
        assert np.abs(d2).max() <= 1e-12 * sc
    t1, t2 = base.copy(), base.copy()
    t1[6] += 0.2
    t2[6] += 0.4
    mu0, mu1, mu2 = o.mu(base), o.mu(t1), o.mu(t2)
    assert np.abs(mu2 - 2 * mu1 + mu0).max() <= 1e-11 * mu0.max()
    assert np.allclose(mu1 - mu0, 0.2 * b, rtol=1e-10)


def test_tau_mirror_symmetry(small):
    """(gL, gR) -> (-gL, -gR) for tau leaves every cross section unchanged."""
    o, rsp, b = small
    t = th(eLL=0.05, eRR=0.1, tLL=0.2, tRR=-0.1, m2=2.0)
    g_l, g_r = -0.5 + SW2, SW2
    tm = t.copy()
    tm[2] = -2 * g_l - t[2]
    tm[3] = -2 * g_r - t[3]
    a, c = o.mu(t), o.mu(tm)
    assert np.allclose(a, c, rtol=1e-13)
    te = t.copy()
    te[0] = -2 * (0.5 + SW2) - t[0]
    assert not np.allclose(o.mu(te), a, rtol=1e-6)  # e-sector: not a mirror
    te[1] = -2 * SW2 - t[1]
    assert np.allclose(o.mu(te), a, rtol=1e-13)


def test_gradient_vs_central_differences(small):
    o, rsp, b = small
    o.set_data(synth.poisson_data(o.mu(SM), 9), b,
               pull_mean=[0, 0, 0, 0, 0, 1, 1],
               pull_sigma=[0, 0, 0, 0, 0, 0.1, 0.1])
    for t in (th(eLL=0.1, eRR=-0.2, tLL=0.3, tRR=0.05, m2=3.0, f8=1.1,
                 fb=0.9), th(eLL=-0.4, tRR=0.4, m2=0.5)):
        v, g = o.nll_grad(t)
        assert v == pytest.approx(o.nll(t), rel=1e-14)
        # five-point central stencil: O(h^4) truncation, and h large enough
        # that the rounding of a -2lnL of order 1e5 stays below 1e-8
        h = 1e-3
        for i in range(7):
            def f(s):
                tt = t.copy()
                tt[i] += s * h
                return o.nll(tt)
            fd = (8 * (f(1) - f(-1)) - (f(2) - f(-2))) / (12 * h)
            assert g[i] == pytest.approx(fd, rel=1e-7, abs=1e-7)


def test_asimov_minimum(small):
    """Asimov data at theta_inj: the gradient vanishes there and every
    coordinate move raises -2lnL."""
    o, rsp, b = small
    t0 = th(eLL=0.05, m2=9.0)
    o.set_data(o.mu(t0), b)
    v, g = o.nll_grad(t0)
    assert np.abs(g).max() < 1e-7
    for i in range(7):
        for s in (-1e-3, 1e-3):
            t = t0.copy()
            t[i] += s
            assert o.nll(t) > v
