"""Seeded synthetic workloads for the spectral-fit likelihood.

This module builds the *inputs* of the model: binning grids, deposited-energy
species shapes, quenching table, multivariate templates, Poisson draws and
request streams.  It holds none of the likelihood arithmetic (no detector
response, no contraction, no pile-up, no NLL): expected counts that a Poisson
draw needs are passed in from stored tables, and every draw is made species by
species so that no sum over species happens here.

The paper (Sec. 3) fits Borexino energy histograms whose expected counts come
from deposited spectra "calculated priorly" and an analytic response (Eq. 1),
pile-up (Eq. 2) and the TFC / radial / pulse-shape terms (Eqs. 3-4).  Borexino
data are not available, so these shapes stand in for them: allowed beta
spectra, a beta+ spectrum shifted by the annihilation energy, Klein-Nishina
Compton recoil shapes, narrow lines, a flat and an exponential background,
with about 500 photoelectrons per MeV (Sec. 2).
"""
from __future__ import annotations

import copy
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

ME = 0.51099895  # electron mass [MeV]

GAUSS = "gauss"
GG = "gg"
TABLE = "table"
COUNT = "count"


# ---------------------------------------------------------------------------
# Model description (plain container; both the oracle and the HIP library take
# exactly these arrays).
# ---------------------------------------------------------------------------
@dataclass
class ModelDesc:
    kind: str                       # "gauss" or "gg"
    true_edges: np.ndarray          # [T+1] float64, increasing
    reco_edges: np.ndarray          # [N+1] float64, increasing
    spectra: np.ndarray             # [S, T] float64, rows >= 0 (unit sum)
    species: list                   # names, len S
    exposure: float = 1.0
    gg_p: float = 1.25              # generalized-gamma exponent (fixed)
    quench: Optional[np.ndarray] = None   # [T] quenching factor (GG only)
    pu_frac: float = 0.0            # pile-up fraction p
    pu_g: Optional[np.ndarray] = None     # [K] random-trigger spectrum
    pu_float: bool = False          # p is a fit parameter (the last entry of theta)
    win: tuple = (0, 0)             # fit window [j_lo, j_hi) over reco bins
    # multivariate fields (None = single energy histogram)
    tag_frac: Optional[np.ndarray] = None  # [S]
    rad_tmpl: Optional[np.ndarray] = None  # [S, n_rad]
    rad_win: tuple = (0, 0)                # reco window feeding the radial term
    ps_tmpl: Optional[np.ndarray] = None   # [S, n_ps]
    # joint energy x radius x pulse-shape term of the vetoed events instead of
    # the three additive terms (needs both templates; data in Data.joint)
    joint: bool = False
    # tabulated response (kind "table"): matrices R_g [G, N, T] at the grid
    # points lam_g of one response coordinate, interpolated linearly in lam
    table_grid: Optional[np.ndarray] = None  # [G] increasing
    table_R: Optional[np.ndarray] = None     # [G, N, T]
    # parameters
    theta_true: Optional[np.ndarray] = None
    float_mask: Optional[np.ndarray] = None
    param_names: list = field(default_factory=list)

    @property
    def T(self):
        return len(self.true_edges) - 1

    @property
    def N(self):
        return len(self.reco_edges) - 1

    @property
    def S(self):
        return self.spectra.shape[0]

    @property
    def n_resp(self):
        if self.kind == TABLE:
            return 1 if len(self.table_grid) > 1 else 0
        return 2 if self.kind == GAUSS else 4  # the count estimator: L, v0, v1, v2 as the GG

    @property
    def P(self):
        return self.S + self.n_resp + (1 if self.pu_float else 0)

    @property
    def multivariate(self):
        return self.tag_frac is not None

    def copy(self):
        return copy.deepcopy(self)


@dataclass
class Data:
    """Observed histograms (float64 counts)."""
    energy: np.ndarray                    # [N] (TFC-vetoed when multivariate)
    tagged: Optional[np.ndarray] = None   # [N]
    radial: Optional[np.ndarray] = None   # [n_rad]
    ps: Optional[np.ndarray] = None       # [N, n_ps]
    joint: Optional[np.ndarray] = None    # [N, n_rad, n_ps] (joint term)


# ---------------------------------------------------------------------------
# Shape primitives, integrated per true bin with 16-point Gauss-Legendre.
# ---------------------------------------------------------------------------
_GL_X, _GL_W = np.polynomial.legendre.leggauss(16)


def _bin_integrals(edges, density, lo, hi):
    """Integral of density over each bin [e_i, e_i+1) clipped to [lo, hi]."""
    out = np.zeros(len(edges) - 1)
    for i in range(len(edges) - 1):
        a = max(edges[i], lo)
        b = min(edges[i + 1], hi)
        if b <= a:
            continue
        x = 0.5 * (b - a) * _GL_X + 0.5 * (b + a)
        out[i] = 0.5 * (b - a) * float(np.dot(_GL_W, density(x)))
    return out


def beta_shape(edges, q, shift=0.0):
    """Allowed beta spectrum (no Fermi function), endpoint q, offset shift."""
    def dens(e):
        t = np.clip(e - shift, 0.0, q)
        return np.sqrt(t * (t + 2 * ME)) * (t + ME) * (q - t) ** 2
    return _bin_integrals(edges, dens, shift, shift + q)


def compton_shape(edges, eg):
    """Klein-Nishina recoil-electron spectrum of a gamma of energy eg."""
    eps = eg / ME
    tmax = 2 * eg * eg / (ME + 2 * eg)

    def dens(t):
        s = np.clip(t / eg, 0.0, tmax / eg)
        return 2 + s * s / (eps * eps * (1 - s) ** 2) + s / (1 - s) * (s - 2 / eps)
    return _bin_integrals(edges, dens, 0.0, tmax)


def line_shape(edges, e0, sig):
    def dens(e):
        return np.exp(-0.5 * ((e - e0) / sig) ** 2)
    return _bin_integrals(edges, dens, e0 - 12 * sig, e0 + 12 * sig)


def flat_shape(edges):
    return _bin_integrals(edges, lambda e: np.ones_like(e), edges[0], edges[-1])


def exp_shape(edges, scale):
    return _bin_integrals(edges, lambda e: np.exp(-e / scale), edges[0], edges[-1])


def _unit(v):
    return v / v.sum()


def quench_table(true_edges):
    """Birks-like quenching factor at each true-bin centre: 1 - 0.25 exp(-E/0.2)."""
    ec = 0.5 * (true_edges[:-1] + true_edges[1:])
    return 1.0 - 0.25 * np.exp(-ec / 0.2)


# ---------------------------------------------------------------------------
# Configurations.
# ---------------------------------------------------------------------------
def config1() -> ModelDesc:
    """Plain 1D fit: 400 true bins (0-2 MeV, 5 keV), 200 reco bins (10 keV),
    4 species, Gaussian response sigma = sqrt(a E + b E^2), 1e5 events."""
    te = 0.005 * np.arange(401)
    re = 0.010 * np.arange(201)
    shapes = [beta_shape(te, 0.6), beta_shape(te, 1.2), line_shape(te, 0.8, 0.010),
              flat_shape(te)]
    names = ["beta_0.6", "beta_1.2", "line_0.8", "flat"]
    rates = np.array([4e4, 3e4, 2e4, 1e4])
    theta = np.concatenate([rates, [0.05, 0.001]])
    return ModelDesc(kind=GAUSS, true_edges=te, reco_edges=re,
                     spectra=np.array([_unit(s) for s in shapes]), species=names,
                     win=(0, 200), theta_true=theta,
                     float_mask=np.ones(6, dtype=bool),
                     param_names=[f"r_{n}" for n in names] + ["a", "b"])


_C2_SPECIES = [
    ("beta_0.156", lambda te: beta_shape(te, 0.156)),
    ("beta_0.56", lambda te: beta_shape(te, 0.56)),
    ("beta_1.16", lambda te: beta_shape(te, 1.16)),
    ("beta_2.25", lambda te: beta_shape(te, 2.25)),
    ("betaplus_0.96", lambda te: beta_shape(te, 0.96, shift=2 * ME)),
    ("compton_0.6", lambda te: compton_shape(te, 0.6)),
    ("compton_0.862", lambda te: compton_shape(te, 0.862)),
    ("compton_1.442", lambda te: compton_shape(te, 1.442)),
    ("compton_2.0", lambda te: compton_shape(te, 2.0)),
    ("line_0.41", lambda te: line_shape(te, 0.41, 0.005)),
    ("line_1.17", lambda te: line_shape(te, 1.17, 0.005)),
    ("line_1.46", lambda te: line_shape(te, 1.46, 0.005)),
]
_C2_FRAC = [.55, .05, .08, .02, .06, .03, .10, .02, .02, .05, .01, .01]
_C4_EXTRA = [("flat", flat_shape), ("exp_0.5", lambda te: exp_shape(te, 0.5))]
C2_EVENTS = 3e6
# generalized-gamma response at the truth: light yield L [p.e./MeV] and
# resolution s^2 = v0 + v1 m + v2 m^2 [p.e.^2]
C2_RESP = np.array([500.0, 4.0, 1.1, 4e-4])
C2_PU_FRAC = 0.02
C2_PU_K = 128

_shape_cache = {}


def _c2_shapes(te, extra=False):
    key = (len(te), float(te[-1]), extra)
    if key not in _shape_cache:
        sp = [(n, f(te)) for n, f in _C2_SPECIES]
        if extra:
            sp += [(n, f(te)) for n, f in _C4_EXTRA]
        _shape_cache[key] = ([n for n, _ in sp], np.array([_unit(s) for _, s in sp]))
    names, arr = _shape_cache[key]
    return list(names), arr.copy()


def config2(pu_g: Optional[np.ndarray] = None, catalogue: bool = False) -> ModelDesc:
    """Full single fit: 3000 true bins (0-3 MeV, 1 keV) x 900 reco bins
    (1 p.e.), 12 species, generalized-gamma response with light yield, three
    resolution parameters and tabulated quenching, 2 % pile-up, 3e6 events.

    The random-trigger spectrum g is an input table (it is the response applied
    to the low-energy beta shape, produced offline and stored); pass it in.
    catalogue=True appends the flat and exponential species of the toy study.
    """
    te = 0.001 * np.arange(3001)
    re = np.arange(901, dtype=np.float64)
    names, spectra = _c2_shapes(te, extra=catalogue)
    frac = list(_C2_FRAC) + ([0.02, 0.02] if catalogue else [])
    rates = np.array(frac) * C2_EVENTS
    theta = np.concatenate([rates, C2_RESP])
    mask = np.ones(len(theta), dtype=bool)
    mask[len(rates) + 1] = False  # v0 fixed
    return ModelDesc(kind=GG, true_edges=te, reco_edges=re, spectra=spectra,
                     species=names, gg_p=1.25, quench=quench_table(te),
                     pu_frac=C2_PU_FRAC if pu_g is not None else 0.0,
                     pu_g=None if pu_g is None else np.asarray(pu_g, np.float64),
                     win=(0, 900), theta_true=theta, float_mask=mask,
                     param_names=[f"r_{n}" for n in names] + ["L", "v0", "v1", "v2"])


# tabulated (Monte Carlo) response ---------------------------------------------
def mc_response_tables(true_edges, reco_edges, quench, grid_L, n_mc, seed, res=(4.0, 1.1, 4e-4)):
    """Monte Carlo response matrices R_g [G, N, T]: for each light yield L_g
    and true bin i, n_mc events with energies uniform in the bin, light
    m = L_g Q_i E, a gamma-distributed charge of mean m and variance
    v0 + v1 m + v2 m^2, histogrammed over the reco bins and divided by n_mc
    (charges outside the reco range are lost).  The stand-in for a detector
    simulation's response tables; seeded."""
    rng = np.random.default_rng(seed)
    te = np.asarray(true_edges, np.float64)
    re = np.asarray(reco_edges, np.float64)
    T, N = len(te) - 1, len(re) - 1
    q = np.asarray(quench, np.float64)
    v0, v1, v2 = res
    out = np.zeros((len(grid_L), N, T))
    for g, L in enumerate(grid_L):
        E = te[:-1, None] + (te[1:] - te[:-1])[:, None] * rng.random((T, n_mc))
        m = L * q[:, None] * E
        s2 = v0 + v1 * m + v2 * m * m
        x = rng.gamma(m * m / s2, s2 / m)
        j = np.searchsorted(re, x, side="right") - 1
        ok = (j >= 0) & (j < N)
        col = np.broadcast_to(np.arange(T)[:, None], j.shape)
        np.add.at(out[g], (j[ok], col[ok]), 1.0)
        out[g] /= n_mc
    return out


def table_config(grid_L=(480.0, 490.0, 500.0, 510.0, 520.0), n_mc=4000, seed=17,
                 true_step=0.001, reco_step=1.0, pu_g: Optional[np.ndarray] = None) -> ModelDesc:
    """The config-2 species and binning (or coarser grids) with a tabulated
    response: Monte Carlo matrices at the light yields grid_L, the fit
    coordinate being the light yield.  theta = rates, L (then the pile-up
    fraction when it floats)."""
    te = true_step * np.arange(int(round(3.0 / true_step)) + 1)
    re = reco_step * np.arange(int(round(900 / reco_step)) + 1)
    names, spectra = _c2_shapes(te)
    q = quench_table(te)
    R = mc_response_tables(te, re, q, grid_L, n_mc, seed)
    rates = np.array(_C2_FRAC) * C2_EVENTS
    grid = np.asarray(grid_L, np.float64)
    theta = np.concatenate([rates, [0.5 * (grid[len(grid) // 2 - 1] + grid[len(grid) // 2])] if len(grid) > 1 else []])
    return ModelDesc(kind=TABLE, true_edges=te, reco_edges=re, spectra=spectra, species=names,
                     pu_frac=C2_PU_FRAC if pu_g is not None else 0.0,
                     pu_g=None if pu_g is None else np.asarray(pu_g, np.float64),
                     win=(0, len(re) - 1), table_grid=grid, table_R=R, theta_true=theta,
                     float_mask=np.ones(len(theta), dtype=bool),
                     param_names=[f"r_{n}" for n in names] + (["L"] if len(grid) > 1 else []))


# count estimator (number of fired PMTs) -------------------------------------
# light yield in fired PMTs per MeV and the count variance v0 + v1 m + v2 m^2
# (v1 = 1: Poisson, v0 and v2 the extra spread)
COUNT_RESP = np.array([300.0, 2.0, 1.0, 2e-3])


def count_config(T=3000, N=1000) -> ModelDesc:
    """The config-2 species measured by a second, discrete estimator: the
    number of fired PMTs, one reco bin per count value 0..N-1."""
    te = (3.0 / T) * np.arange(T + 1)
    re = np.arange(N + 1, dtype=np.float64)
    names, spectra = _c2_shapes(te)
    rates = np.array(_C2_FRAC) * C2_EVENTS
    theta = np.concatenate([rates, COUNT_RESP])
    mask = np.ones(len(theta), dtype=bool)
    mask[len(rates) + 1] = False  # v0 fixed
    return ModelDesc(kind=COUNT, true_edges=te, reco_edges=re, spectra=spectra, species=names,
                     quench=quench_table(te), win=(0, N), theta_true=theta, float_mask=mask,
                     param_names=[f"r_{n}" for n in names] + ["L", "v0", "v1", "v2"])


def count_events(d: ModelDesc, theta, seed=0) -> Data:
    """A histogram of the count estimator from simulated events: for each
    species a Poisson number of events (mean r_s), true energies from its
    deposited spectrum, fired-PMT counts drawn around L Q E with the
    variance v0 + v1 m + v2 m^2 (negative binomial); counts beyond the
    reco range are lost."""
    rng = np.random.default_rng(seed)
    te = np.asarray(d.true_edges, np.float64)
    ec = 0.5 * (te[:-1] + te[1:])
    L, v0, v1, v2 = np.asarray(theta, np.float64)[d.S:d.S + 4]
    hist = np.zeros(d.N)
    for s in range(d.S):
        n_ev = rng.poisson(theta[s])
        i = rng.choice(len(ec), size=n_ev, p=d.spectra[s] / d.spectra[s].sum())
        m = L * np.asarray(d.quench)[i] * ec[i]
        s2 = v0 + v1 * m + v2 * m * m
        r = m * m / (s2 - m)
        c = rng.negative_binomial(r, r / (r + m))
        j = c - int(d.reco_edges[0])
        ok = (j >= 0) & (j < d.N)
        hist += np.bincount(j[ok], minlength=d.N)[: d.N]
    return Data(energy=hist)


def joint_events(d: ModelDesc, theta, seed=0) -> Data:
    """Simulated histograms of a multivariate generalized-gamma model with the
    joint term: per species a Poisson number of events, true energies from
    its spectrum, a gamma-distributed charge around L Q E with variance
    v0 + v1 m + v2 m^2 (1 p.e. reco bins), tagged with probability t_s (the
    tagged energy histogram), else a radial bin from rho_s and a pulse-shape
    bin from T_s (the joint histogram).  A stand-in for a detector
    simulation, seeded."""
    rng = np.random.default_rng(seed)
    te = np.asarray(d.true_edges, np.float64)
    ec = 0.5 * (te[:-1] + te[1:])
    th = np.asarray(theta, np.float64)
    L, v0, v1, v2 = th[d.S:d.S + 4]
    n_rad, n_ps = d.rad_tmpl.shape[1], d.ps_tmpl.shape[1]
    joint = np.zeros((d.N, n_rad, n_ps))
    tagged = np.zeros(d.N)
    for s in range(d.S):
        n_ev = rng.poisson(th[s])
        i = rng.choice(len(ec), size=n_ev, p=d.spectra[s] / d.spectra[s].sum())
        m = L * np.asarray(d.quench)[i] * ec[i]
        s2 = v0 + v1 * m + v2 * m * m
        q = rng.gamma(m * m / s2, s2 / m)
        j = np.searchsorted(d.reco_edges, q, side="right") - 1
        ok = (j >= 0) & (j < d.N)
        tag = rng.random(n_ev) < d.tag_frac[s]
        tagged += np.bincount(j[ok & tag], minlength=d.N)[: d.N]
        v = ok & ~tag
        k = rng.choice(n_rad, size=int(v.sum()), p=d.rad_tmpl[s] / d.rad_tmpl[s].sum())
        l = rng.choice(n_ps, size=int(v.sum()), p=d.ps_tmpl[s] / d.ps_tmpl[s].sum())
        np.add.at(joint, (j[v], k, l), 1.0)
    return Data(energy=None, tagged=tagged, joint=joint)


# multivariate templates ------------------------------------------------------
N_RAD = 100
N_PS = 50


def radial_templates(external):
    """100 radial bins on [0, 3) m. Internal: uniform in volume; external:
    density r^2 exp((r-3)/0.5)."""
    re = np.linspace(0.0, 3.0, N_RAD + 1)
    internal = _unit(re[1:] ** 3 - re[:-1] ** 3)
    ext = _unit(_bin_integrals(re, lambda r: r * r * np.exp((r - 3.0) / 0.5), 0.0, 3.0))
    return np.array([ext if e else internal for e in external])


def ps_templates(betaplus):
    """50 pulse-shape bins on [0, 1): Gaussian of width 0.1 centred at 0.6
    (beta+) or 0.4 (others), integrated per bin by quadrature."""
    pe = np.linspace(0.0, 1.0, N_PS + 1)
    out = []
    for bp in betaplus:
        c = 0.6 if bp else 0.4
        out.append(_unit(_bin_integrals(pe, lambda x: np.exp(-0.5 * ((x - c) / 0.1) ** 2), 0, 1)))
    return np.array(out)


def _make_mv(d: ModelDesc, betaplus_idx, external_idx) -> ModelDesc:
    S = d.S
    t = np.zeros(S)
    t[list(betaplus_idx)] = 0.9
    d.tag_frac = t
    d.rad_tmpl = radial_templates([s in external_idx for s in range(S)])
    d.rad_win = (0, d.N)
    d.ps_tmpl = ps_templates([s in betaplus_idx for s in range(S)])
    return d


def config3a() -> ModelDesc:
    """Multivariate fit on the config-1 model (PS histogram 200 x 50)."""
    return _make_mv(config1(), betaplus_idx=[1], external_idx=[3])


def config3b(pu_g: Optional[np.ndarray] = None) -> ModelDesc:
    """Multivariate fit on the config-2 model (PS histogram 900 x 50)."""
    return _make_mv(config2(pu_g), betaplus_idx=[4], external_idx=[8, 11])


# ---------------------------------------------------------------------------
# Poisson draws.  `per_species` holds stored expected counts per unit rate
# (one column per species); each species is drawn on its own and the counts
# added, which has the law of a single Poisson draw of the total.
# ---------------------------------------------------------------------------
def draw_species_sum(rng, per_species, rates):
    out = np.zeros(per_species.shape[:-1])
    for s, r in enumerate(rates):
        out += rng.poisson(r * per_species[..., s])
    return out.astype(np.float64)


def draw_poisson(rng, mu):
    return rng.poisson(mu).astype(np.float64)


# ---------------------------------------------------------------------------
# Config 4: ragged toy catalogue.
# ---------------------------------------------------------------------------
@dataclass
class Toy:
    index: int
    n_reco: int
    n_species: int
    theta_true: np.ndarray
    theta0: np.ndarray
    counts: np.ndarray
    species: np.ndarray   # catalogue indices of the floated species


# A species is floated in a toy only if its expectation inside the toy's reco
# window is at least this many events: a species with (numerically) nothing in
# the window leaves its rate unconstrained, and the fit of such a toy is not
# well posed.
TOY_MIN_EVENTS = 1000.0


def toy_shape(b):
    rng = np.random.default_rng([4, b])
    n_reco = int(rng.integers(300, 901))
    n_species = int(rng.integers(6, 15))
    return rng, n_reco, n_species


def toy_species(n_reco, n_species, per_species_catalogue, theta_cat):
    """The first n_species catalogue species (in catalogue order) with at
    least TOY_MIN_EVENTS expected events in reco bins [0, n_reco)."""
    n_cat = per_species_catalogue.shape[1]
    inside = per_species_catalogue[:n_reco].sum(0) * theta_cat[:n_cat]
    ok = np.flatnonzero(inside >= TOY_MIN_EVENTS)
    return ok[:n_species]


def toy(b, per_species_catalogue, theta_cat) -> Toy:
    """Toy b of the batched study.  per_species_catalogue: stored expected
    counts per unit rate, [900, 14], of the catalogue model at the truth."""
    rng, n_reco, n_species = toy_shape(b)
    sp = toy_species(n_reco, n_species, per_species_catalogue, theta_cat)
    n_species = len(sp)
    rates = theta_cat[sp].copy()
    resp = theta_cat[-4:].copy()
    counts = draw_species_sum(rng, per_species_catalogue[:n_reco, sp], rates)
    theta_true = np.concatenate([rates, resp])
    z = rng.standard_normal(len(theta_true))
    theta0 = theta_true * (1 + 0.05 * z)
    theta0[:n_species] = np.maximum(theta0[:n_species], 1.0)
    theta0[n_species + 1] = theta_true[n_species + 1]  # v0 is fixed
    return Toy(b, n_reco, n_species, theta_true, theta0, counts, sp)


def toy_desc(base_catalogue: ModelDesc, t: Toy) -> ModelDesc:
    d = base_catalogue.copy()
    d.reco_edges = d.reco_edges[: t.n_reco + 1].copy()
    d.spectra = d.spectra[t.species].copy()
    d.species = [d.species[i] for i in t.species]
    d.win = (0, t.n_reco)
    d.theta_true = t.theta_true.copy()
    mask = np.ones(t.n_species + 4, dtype=bool)
    mask[t.n_species + 1] = False
    d.float_mask = mask
    d.param_names = [f"r_{n}" for n in d.species] + ["L", "v0", "v1", "v2"]
    return d


# ---------------------------------------------------------------------------
# Config 5: request stream.
# ---------------------------------------------------------------------------
@dataclass
class Request:
    t_arrival: float   # seconds from stream start
    kind: str          # "fit1", "fit2" or "evalgrad"


def request_stream(qps, n=2000):
    rng = np.random.default_rng([5, int(qps)])
    gaps = rng.exponential(1.0 / qps, size=n)
    u = rng.random(n)
    kinds = np.where(u < 0.45, "fit1", np.where(u < 0.90, "fit2", "evalgrad"))
    t = np.cumsum(gaps)
    return [Request(float(a), str(k)) for a, k in zip(t, kinds)], rng


# ---------------------------------------------------------------------------
# Frozen datasets (written offline into tests/golden by make_fixtures.py).
# ---------------------------------------------------------------------------
GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "tests", "golden")


def _npz(name):
    return np.load(os.path.join(GOLDEN, name + ".npz"))


def load(name):
    """(ModelDesc, Data) for "c1", "c2", "c3a" or "c3b" at the frozen data."""
    if name == "c1":
        z = _npz("c1")
        return config1(), Data(energy=z["energy"])
    g = _npz("c2")["pu_g"]
    if name == "c2":
        return config2(pu_g=g), Data(energy=_npz("c2")["energy"])
    if name in ("c3a", "c3b"):
        z = _npz(name)
        d = config3a() if name == "c3a" else config3b(g)
        return d, Data(energy=z["sub"], tagged=z["tag"], radial=z["radial"], ps=z["ps"])
    raise KeyError(name)


def pileup_spectrum():
    return _npz("c2")["pu_g"]


def catalogue():
    """(ModelDesc of the 14-species toy catalogue, per-species expectations
    [900, 14], theta at the truth)."""
    z = _npz("c4")
    return config2(pu_g=pileup_spectrum(), catalogue=True), z["per_species"], z["theta"]


def species_table(name):
    """Stored per-unit-rate expectations used for fresh Poisson draws."""
    if name == "c1":
        return _npz("c1")["per_species"]
    if name == "c2":
        return _npz("c4")["per_species"][:, :12]
    raise KeyError(name)
