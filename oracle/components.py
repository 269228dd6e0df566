"""Multi-component likelihood (test infrastructure only; shares nothing with
the library).

Written from Sec. III.B-C literally, in FP64:
  Eq. (Rij):          R^(k)_ij = (N^(k)_ij / M^(k)_j) / sum (N / M) * s^(k)
                      (then stored in FP32, as the library stores every
                      response)
  Eq. (fNp_reweight): f^(k)_Np(j) = 1 / sum_l f^(k)_T(T_l)
                                    * sum_i R^(k)_ij f^(k)_T(T_i) / fhat^SM,(k)(T_i)
  Eq. (mu_total):     mu_j = MT M_j [ sum_k rate_k f^(k)_Np(j) + sum_b r_b Rate_b pdf_b(j) ]
  Eq. (logL):         -2lnL = 2 sum_j [mu_j - n_j ln mu_j + lnGamma(n_j+1)] + pulls
with the reading that a signal rate carries its integrated cross section,
rate_k = r_k Rate_k sum_l f^(k)_T(T_l; theta) / sum_l f^(k)_T(T_l; SM), and
f_T / fhat^SM := sum_l f^SM_T(T_l) where the SM spectrum is zero (the weight
one of the single-component form).  The recoil spectra f^(k)_T come from one
single-component oracle per component holding that component's sources.
Parameter vector: [eps_eL, eps_eR, eps_tauL, eps_tauR, m2, r_1..r_K, r_b1..r_bB].
"""
from __future__ import annotations

import math

import numpy as np

from . import Oracle


class ComponentOracle:
    def __init__(self, sources, comp_of_source, n_t, hist, scale, rate_sm,
                 bkg_pdf=None, bkg_rate=None, comp_mask=None, mask=None,
                 exposure=1.0, t_hi=16.0):
        hist = np.asarray(hist, dtype=np.float64)
        self.K, self.n_t, self.n_reco = hist.shape
        self.B = 0 if bkg_pdf is None else len(bkg_pdf)
        self.orc = []
        for k in range(self.K):
            o = Oracle()
            o.set_sources([dict(s, group=0) for s, c in zip(sources, comp_of_source)
                           if c == k], n_t, 0.0, t_hi)
            self.orc.append(o)
        self.R = []
        for k in range(self.K):
            M = np.ones(self.n_reco) if comp_mask is None else np.asarray(comp_mask[k], float)
            NM = np.where(hist[k] > 0, hist[k] / M[None, :], 0.0)
            Rk = NM / NM.sum() * float(scale[k])
            self.R.append(Rk.astype(np.float32).astype(np.float64))
        self.rate_sm = np.asarray(rate_sm, dtype=np.float64)
        self.bkg = (np.zeros((0, self.n_reco)) if self.B == 0 else
                    np.asarray(bkg_pdf, float) * np.asarray(bkg_rate, float)[:, None])
        self.mask = np.ones(self.n_reco) if mask is None else np.asarray(mask, float)
        self.MT = float(exposure)
        std_sm = np.array([0, 0, 0, 0, 0, 1.0, 1.0])
        self.fsm = [o.spectrum(std_sm) for o in self.orc]
        self.n = None
        self.n_theta = 5 + self.K + self.B

    def set_data(self, n, pull_mean=None, pull_sigma=None):
        self.n = np.asarray(n, dtype=np.float64)
        self.pm = None if pull_mean is None else np.asarray(pull_mean, float)
        self.ps = None if pull_sigma is None else np.asarray(pull_sigma, float)

    def f_np(self, k, theta):
        """Eq. (fNp_reweight) for component k and the rate factor
        sum f_T / sum f_T^SM of the reading."""
        std = np.concatenate([np.asarray(theta[:5], float), [1.0, 1.0]])
        f = self.orc[k].spectrum(std)
        fsm = self.fsm[k]
        fhat = fsm / fsm.sum()
        ratio = np.where(fhat > 0, f / np.where(fhat > 0, fhat, 1.0), fsm.sum())
        fnp = (self.R[k] * ratio[:, None]).sum(0) / f.sum()
        return fnp, f.sum() / fsm.sum()

    def mu(self, theta):
        theta = np.asarray(theta, dtype=np.float64)
        s = np.zeros(self.n_reco)
        for k in range(self.K):
            fnp, share = self.f_np(k, theta)
            rate = theta[5 + k] * self.rate_sm[k] * share
            s += rate * fnp
        for b in range(self.B):
            s += theta[5 + self.K + b] * self.bkg[b]
        return self.MT * self.mask * s

    def nll(self, theta):
        mu = self.mu(theta)
        n = self.n
        if np.any((mu <= 0) & (n > 0)):
            return math.inf
        t = mu - np.where(n > 0, n * np.log(np.where(mu > 0, mu, 1.0)), 0.0)
        lg = np.array([math.lgamma(x + 1.0) for x in n])
        v = 2.0 * float(np.sum(t + lg))
        if self.pm is not None:
            th = np.asarray(theta, dtype=np.float64)
            on = self.ps > 0
            v += float(np.sum(((th[on] - self.pm[on]) / self.ps[on]) ** 2))
        return v

    def close(self):
        for o in self.orc:
            o.close()
