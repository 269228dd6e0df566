"""Closure of the bin-level reweighting against a direct continuum fold
(Sec. VI.A of the paper; test infrastructure only).

A single 7Be line, an analytic scintillator response (light yield Y
photoelectrons per MeV, a quenching non-linearity that lowers the yield at
low energy, Gaussian photo-statistics with variance equal to the mean) and
two predictions of the N_p spectrum:

  direct      sum_i  int_{bin i} S_theta(T) P(j | T) dT
  reweighted  sum_i [int_{bin i} S_SM(T) P(j | T) dT] * S_theta(T_i)/S_SM(T_i)

with T_i the bin centre.  Both use the same Gauss-Legendre rule inside each
recoil bin, so their difference is exactly the single-representative-energy
approximation of the weights.  S is the flavour-summed cross section of the
oracle (Eqs. (sm_cross_section), (xs_nsi), (xs_mm), (xs_total)).

Readings: the quench is N(T) = Y T^2/(T + T_q) with T_q = 0.05 MeV (the
paper states only that quenching lowers the low-energy yield); the recoil
grid spans [0, T_max] of the line; N_p bins are 1 photoelectron wide.
"""
import math

import numpy as np
from scipy import special

from . import Oracle

BE7 = 0.862
ME = 0.51099895


def line_tmax(E):
    return 2 * E * E / (ME + 2 * E)


def mean_pe(T, Y=500.0, Tq=0.05):
    return Y * T * T / (T + Tq)


def spectrum(o, E, Ts, theta, pee):
    P = (pee, (1 - pee) / 2, (1 - pee) / 2)
    return np.array([sum(P[a] * o.dsigma(a, E, T, theta) for a in range(3))
                     for T in Ts])


def response_rows(Ts, edges):
    """P(N_p in [edges_j, edges_j+1) | T) for every T (Gaussian, var = mean)."""
    nb = mean_pe(Ts)[:, None]
    s = np.sqrt(nb)
    c = special.ndtr((edges[None, :] - nb) / s)
    return np.diff(c, axis=1)


def predictions(theta, n_t, edges, E=BE7, n_gl=16):
    o = Oracle()
    pee = 0.32 + 0.23 / (1 + (E / 2) ** 2)
    tmax = line_tmax(E)
    xg, wg = np.polynomial.legendre.leggauss(n_gl)
    dt = tmax / n_t
    centres = (np.arange(n_t) + 0.5) * dt
    sm = np.array([0, 0, 0, 0, 0, 1, 1], dtype=float)
    # quadrature nodes inside every recoil bin
    Tn = (centres[:, None] + 0.5 * dt * xg[None, :]).ravel()
    Wn = np.tile(0.5 * dt * wg, n_t)
    s_sm = spectrum(o, E, Tn, sm, pee)
    s_th = spectrum(o, E, Tn, theta, pee)
    Pj = response_rows(Tn, edges)
    direct = ((Wn * s_th)[:, None] * Pj).reshape(n_t, n_gl, -1).sum(1).sum(0)
    Rjoint = ((Wn * s_sm)[:, None] * Pj).reshape(n_t, n_gl, -1).sum(1)
    w = spectrum(o, E, centres, theta, pee) / spectrum(o, E, centres, sm, pee)
    reweighted = (Rjoint * w[:, None]).sum(0)
    return direct, reweighted


def binned_response(n_t, edges, E=BE7, n_gl=16):
    """The reweighting's fixed inputs: the joint SM response of each recoil
    bin [n_t][n_bins] (integral over the bin of S_SM(T) P(j | T)), the line's
    survival probability and the recoil range."""
    o = Oracle()
    pee = 0.32 + 0.23 / (1 + (E / 2) ** 2)
    tmax = line_tmax(E)
    xg, wg = np.polynomial.legendre.leggauss(n_gl)
    dt = tmax / n_t
    centres = (np.arange(n_t) + 0.5) * dt
    sm = np.array([0, 0, 0, 0, 0, 1, 1], dtype=float)
    Tn = (centres[:, None] + 0.5 * dt * xg[None, :]).ravel()
    Wn = np.tile(0.5 * dt * wg, n_t)
    s_sm = spectrum(o, E, Tn, sm, pee)
    Pj = response_rows(Tn, edges)
    Rjoint = ((Wn * s_sm)[:, None] * Pj).reshape(n_t, n_gl, -1).sum(1)
    return Rjoint, pee, tmax


def closure(theta, n_t, lo=50, hi=400):
    """(max bin-by-bin relative residual, integral relative deviation) over
    lo < N_p < hi."""
    edges = np.arange(0.0, 451.0)
    d, r = predictions(theta, n_t, edges)
    sel = (edges[:-1] >= lo) & (edges[1:] <= hi)
    bin_res = float(np.max(np.abs(r[sel] - d[sel]) / d[sel]))
    integ = float(abs(r[sel].sum() - d[sel].sum()) / d[sel].sum())
    return bin_res, integ
