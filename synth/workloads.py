"""Seeded synthetic workloads for the spectrum-reweighting likelihood.

Everything here is an *input* to the method:

* solar source tables -- energy nodes, per-node weight phi(E)*dE (or the
  line flux), the survival probability P_ee at each node and a group flag
  (1 = scaled by the 8B flux normalisation);
* the detector response R_cond[T, E_reco], histogrammed from a seeded
  Monte Carlo of mono-energetic recoil electrons whose true kinetic energy
  is drawn flat in T (the "flatter recoil spectrum" sampling the paper
  recommends for low-recoil support, Sec. VI.A last paragraph), with a
  Birks-like quench and Gaussian photo-statistics smearing;
* Poisson data drawn from an expectation the *caller* provides;
* parameter-point lists.

Parameter vector layout (7 doubles per point):
    theta = [eps_eL, eps_eR, eps_tauL, eps_tauR, m2, f_8B, f_bkg]
with m2 = (mu_nu / 1e-11 mu_B)^2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "T_LO", "T_HI", "RECO_LO", "RECO_HI", "N_THETA", "SOURCES",
    "survival_prob", "beta_shape", "source_nodes", "response_mc",
    "poisson_data", "theta_prior", "theta_corners", "theta_sm",
    "theta_grid_scan", "theta_box", "Config", "CONFIGS", "batched_schedule",
    "rng", "component_inputs",
]

T_LO, T_HI = 0.0, 16.0          # recoil-energy histogram range [MeV]
RECO_LO, RECO_HI = 0.0, 16.0    # reconstructed-energy histogram range [MeV]
N_THETA = 7

# name, kind ("beta" continuum or "line"), endpoint / line energy [MeV],
# flux [cm^-2 s^-1] (only the ratios matter), group (1 = scaled by f_8B)
SOURCES = (
    ("pp", "beta", 0.42, 6.0e10, 0),
    ("7Be", "line", 0.862, 4.5e9, 0),
    ("pep", "line", 1.44, 1.4e8, 0),
    ("CNO", "beta", 1.73, 4.9e8, 0),
    ("8B", "beta", 16.0, 5.5e6, 1),
)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def survival_prob(E):
    """Electron-neutrino survival probability used by every workload."""
    E = np.asarray(E, dtype=np.float64)
    return 0.32 + 0.23 / (1.0 + (E / 2.0) ** 2)


def beta_shape(E, E0):
    """Unit-normalised allowed beta shape 30 E^2 (E0-E)^2 / E0^5 on [0, E0]."""
    E = np.asarray(E, dtype=np.float64)
    return 30.0 * E * E * (E0 - E) ** 2 / E0 ** 5


def source_nodes(n_e: int, sources=SOURCES):
    """Node tables: continua on n_e midpoint nodes with rectangle weights,
    lines as a single node carrying the line flux."""
    out = []
    for name, kind, e0, flux, group in sources:
        if kind == "beta":
            de = e0 / n_e
            E = (np.arange(n_e, dtype=np.float64) + 0.5) * de
            wgt = flux * beta_shape(E, e0) * de
            k = 1
        else:
            E = np.array([e0], dtype=np.float64)
            wgt = np.array([flux], dtype=np.float64)
            k = 0
        out.append(dict(name=name, kind=k, E=E, weight=wgt,
                        p_ee=survival_prob(E), group=int(group)))
    return out


@dataclass
class Response:
    R: np.ndarray            # float32 [n_t, n_reco], conditional response
    counts: np.ndarray       # int64   [n_t, n_reco]
    row_events: np.ndarray   # int64   [n_t] events generated per true bin
    under: np.ndarray        # int64   [n_t] E_vis < RECO_LO
    over: np.ndarray         # int64   [n_t] E_vis >= RECO_HI
    n_events: int


def response_mc(n_t: int, n_reco: int, n_events: int, seed: int,
                kb: float = 0.01, res: float = 0.05,
                chunk: int = 1 << 23, keep_counts: bool = True) -> Response:
    """Histogram a flat-in-T electron Monte Carlo into R_cond[T, E_reco].

    Each event: T ~ U(T_LO, T_HI); quenched light Q = T / (1 + kb T);
    E_vis = Q + res * sqrt(Q / MeV) * MeV * z with z ~ N(0, 1).
    R_cond[l, j] = N_lj / N_l, so each row sums to the detection efficiency
    (events outside [RECO_LO, RECO_HI) are counted in under/over).
    """
    g = rng(seed)
    dt = (T_HI - T_LO) / n_t
    dr = (RECO_HI - RECO_LO) / n_reco
    nbin = n_t * n_reco
    counts = np.zeros(nbin, dtype=np.int64)
    row_events = np.zeros(n_t, dtype=np.int64)
    under = np.zeros(n_t, dtype=np.int64)
    over = np.zeros(n_t, dtype=np.int64)
    left = int(n_events)
    while left > 0:
        m = min(chunk, left)
        left -= m
        T = g.uniform(T_LO, T_HI, m)
        z = g.standard_normal(m)
        l = np.minimum(((T - T_LO) / dt).astype(np.int64), n_t - 1)
        Q = T / (1.0 + kb * T)
        ev = Q + res * np.sqrt(Q) * z
        row_events += np.bincount(l, minlength=n_t)
        lo = ev < RECO_LO
        hi = ev >= RECO_HI
        under += np.bincount(l[lo], minlength=n_t)
        over += np.bincount(l[hi], minlength=n_t)
        ok = ~(lo | hi)
        j = np.minimum(((ev[ok] - RECO_LO) / dr).astype(np.int64), n_reco - 1)
        counts += np.bincount(l[ok] * n_reco + j, minlength=nbin)
    counts = counts.reshape(n_t, n_reco)
    denom = np.where(row_events > 0, row_events, 1).astype(np.float64)
    R = (counts / denom[:, None]).astype(np.float32)
    return Response(R=R, counts=counts if keep_counts else None,
                    row_events=row_events, under=under, over=over,
                    n_events=int(n_events))


def poisson_data(mu, seed: int) -> np.ndarray:
    """Binned data n_j ~ Poisson(mu_j), returned as float64."""
    return rng(seed).poisson(np.asarray(mu, dtype=np.float64)).astype(np.float64)


def theta_sm() -> np.ndarray:
    return np.array([0, 0, 0, 0, 0, 1, 1], dtype=np.float64)


def theta_prior(n: int, seed: int, f_range=None) -> np.ndarray:
    """eps_{e,tau}^{L,R} ~ U(-1/2, 1/2), mu_nu ~ U(0, 5e-11 mu_B);
    f_8B, f_bkg = 1 or ~ U(f_range)."""
    g = rng(seed)
    th = np.empty((n, N_THETA))
    th[:, 0:4] = g.uniform(-0.5, 0.5, (n, 4))
    mu = g.uniform(0.0, 5e-11, n)
    th[:, 4] = (mu / 1e-11) ** 2
    if f_range is None:
        th[:, 5:7] = 1.0
    else:
        th[:, 5:7] = g.uniform(f_range[0], f_range[1], (n, 2))
    return th


def theta_corners() -> np.ndarray:
    """The 2^5 corners of the physics box (eps = +-1/2, mu_nu in {0, 5e-11})."""
    rows = []
    for bits in range(32):
        e = [0.5 if (bits >> i) & 1 else -0.5 for i in range(4)]
        m2 = 25.0 if (bits >> 4) & 1 else 0.0
        rows.append(e + [m2, 1.0, 1.0])
    return np.array(rows, dtype=np.float64)


def theta_grid_scan(p: int, seed: int) -> np.ndarray:
    """(eps_eL, eps_eR) on a 2^ceil(log2 sqrt p) x 2^floor(log2 sqrt p) grid
    over [-1/2, 1/2]^2, mu_nu ~ U(0, 5e-11), everything else nominal."""
    lg = int(round(math.log2(p)))
    na, nb = 2 ** ((lg + 1) // 2), 2 ** (lg // 2)
    assert na * nb == p
    a = np.linspace(-0.5, 0.5, na)
    b = np.linspace(-0.5, 0.5, nb)
    A, B = np.meshgrid(a, b, indexing="ij")
    th = np.zeros((p, N_THETA))
    th[:, 0] = A.ravel()
    th[:, 1] = B.ravel()
    th[:, 4] = (rng(seed).uniform(0.0, 5e-11, p) / 1e-11) ** 2
    th[:, 5:7] = 1.0
    return th


def theta_box():
    """Box the surrogate is trained on: lower and upper bounds per component."""
    lo = np.array([-0.5, -0.5, -0.5, -0.5, 0.0, 0.8, 0.8])
    hi = np.array([0.5, 0.5, 0.5, 0.5, 25.0, 1.2, 1.2])
    return lo, hi


@dataclass
class Config:
    name: str
    n_t: int
    n_reco: int
    n_e: int
    n_mc: int
    n_sig: float = 1.0e4
    bkg: float = 10.0
    seed_base: int = 0
    extra: dict = field(default_factory=dict)

    def seeds(self, d: int = 0):
        c = self.seed_base
        return dict(response=1000 * c + d, data=2000 * c + d,
                    theta=3000 * c + d)


CONFIGS = {
    0: Config("parity-512x256", 512, 256, 256, 10 ** 6, seed_base=0),
    1: Config("paper-scale-16384x4096", 16384, 4096, 2048, 10 ** 8,
              seed_base=1),
    3: Config("gradient-16384x4096", 16384, 4096, 2048, 10 ** 8,
              seed_base=1),
}


def batched_schedule(n_datasets: int = 64):
    """Uneven dataset shapes of the batched scan: N_T = 2048 * 2^(d mod 4),
    N_reco = 512 * 2^(floor(d/4) mod 4), P = 64 * 2^(d mod 7)."""
    out = []
    for d in range(n_datasets):
        out.append(dict(d=d, n_t=2048 * 2 ** (d % 4),
                        n_reco=512 * 2 ** ((d // 4) % 4),
                        n_pts=64 * 2 ** (d % 7), n_e=256, n_mc=10 ** 6,
                        seed_response=1000 * 2 + d, seed_data=2000 * 2 + d,
                        seed_theta=3000 * 2 + d))
    return out


# rough recoil endpoints [MeV] of the five sources (shape parameters of the
# synthetic per-component histograms only) and an exponential slope each
COMPONENT_SHAPES = ((0.26, 0.08), (0.67, 0.3), (1.22, 0.5), (1.52, 0.5),
                    (15.8, 4.0))


def component_inputs(n_t, n_reco, n_mc, seed, shapes=COMPONENT_SHAPES,
                     shared_mc=False):
    """Seeded inputs of the multi-component form: one SM Monte-Carlo
    histogram per component (its own flat-T detector MC, seed + k, or one MC
    shared by all with ``shared_mc``, rows weighted by a falling profile up
    to an endpoint), two background PDFs (flat and falling), per-component
    live-time masks in [0.9, 1] and a common mask with a few dead bins at
    0.5."""
    K = len(shapes)
    T = (np.arange(n_t) + 0.5) * (T_HI - T_LO) / n_t + T_LO
    hist = np.zeros((K, n_t, n_reco), dtype=np.float32)
    rsp = None
    for k, (tend, tau) in enumerate(shapes):
        if rsp is None or not shared_mc:
            rsp = response_mc(n_t, n_reco, n_mc, seed=seed + k, keep_counts=False)
        prof = np.where(T < tend, np.exp(-T / tau), 0.0)
        hist[k] = (rsp.R * (n_mc / n_t) * prof[:, None]).astype(np.float32)
    g = rng(seed + 100)
    E = (np.arange(n_reco) + 0.5) * (RECO_HI - RECO_LO) / n_reco + RECO_LO
    flat = np.full(n_reco, 1.0 / n_reco)
    fall = np.exp(-E / 2.0)
    fall /= fall.sum()
    comp_mask = g.uniform(0.9, 1.0, (K, n_reco))
    mask = np.ones(n_reco)
    mask[g.choice(n_reco, size=max(1, n_reco // 64), replace=False)] = 0.5
    return dict(hist=hist, comp_of_source=np.arange(K, dtype=np.int32),
                scale=g.uniform(0.8, 1.2, K), rate_sm=np.array([1.3e3, 5.0e2, 3.0e1, 6.0e1, 4.0e1]),
                bkg_pdf=np.vstack([flat, fall]), bkg_rate=np.array([2.0e3, 8.0e2]),
                comp_mask=comp_mask, mask=mask, exposure=1.5)
