"""FP64 oracle of the expected counts and the binned Poisson NLL.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline import this.  Everything is materialised and evaluated densely in
float64 with library primitives (scipy.special, numpy matmul / convolve,
math.fsum); there is no tiling, fusion or reordering.

Notation: T true-energy bins with centres E_i, N reco bins with edges x_j,
S species with deposited spectra F[s, i] (unit row sums), rates r_s,
response parameters rho, cells R[j, i] = probability that an event deposited
in true bin i is reconstructed in reco bin j (Eq. 1 discretised).
"""
from __future__ import annotations

import math
from types import SimpleNamespace

import numpy as np
from scipy import special, stats

GAUSS = "gauss"
GG = "gg"
TABLE = "table"
COUNT = "count"


class DomainError(ValueError):
    """Parameters outside the model's domain (the NLL is +inf there)."""


# ---------------------------------------------------------------------------
# Column parameters of the response (Eq. 1: R_x(N_x, E; p0, p1, ...)).
# ---------------------------------------------------------------------------
def true_centres(desc):
    te = np.asarray(desc.true_edges, np.float64)
    return 0.5 * (te[:-1] + te[1:])


def gg_log_cv2(k, p):
    """ln(1 + Var/Mean^2) of the generalized gamma with shape k, exponent p:
    ln[Gamma(k) Gamma(k + 2/p) / Gamma(k + 1/p)^2]."""
    return special.gammaln(k) + special.gammaln(k + 2.0 / p) - 2.0 * special.gammaln(k + 1.0 / p)


def gg_solve_shape(tau, p):
    """Shape k with gg_log_cv2(k, p) = tau, by bisection on ln k (the left
    side decreases monotonically in k)."""
    tau = np.asarray(tau, np.float64)
    lo = np.full(tau.shape, -40.0)
    hi = np.full(tau.shape, 25.0)
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        too_small_k = gg_log_cv2(np.exp(mid), p) > tau
        lo = np.where(too_small_k, mid, lo)
        hi = np.where(too_small_k, hi, mid)
    return np.exp(0.5 * (lo + hi))


def table_cell(desc, resp):
    """Tabulated response: the grid cell [lam_g, lam_g+1] holding the table
    coordinate lam = resp[0] and the weight w of lam_g+1 in the linear
    interpolation.  One grid point: no coordinate (g = 0, w = 0)."""
    grid = np.asarray(desc.table_grid, np.float64)
    if grid.size == 1:
        return 0, 0.0
    lam = float(resp[0])
    if not (grid[0] <= lam <= grid[-1]):
        raise DomainError("table coordinate outside the grid")
    g = int(np.searchsorted(grid, lam, side="right")) - 1
    g = min(max(g, 0), grid.size - 2)
    return g, (lam - grid[g]) / (grid[g + 1] - grid[g])


def column_params(desc, resp):
    """Per true-bin column parameters.

    Gaussian: mean m_i = E_i, sigma_i = sqrt(a E_i + b E_i^2).
    Generalized gamma (Stacy) with fixed exponent p: mean m_i = L Q_i E_i,
    variance s_i^2 = v0 + v1 m_i + v2 m_i^2, and (k_i, a_i) such that
    GG(a, k, p) has that mean and variance:
        Var/Mean^2 = Gamma(k)Gamma(k+2/p)/Gamma(k+1/p)^2 - 1,
        a = m Gamma(k) / Gamma(k + 1/p).
    """
    E = true_centres(desc)
    resp = np.asarray(resp, np.float64)
    if not np.all(np.isfinite(resp)):
        raise DomainError("non-finite response parameter")
    if desc.kind == TABLE:
        g, w = table_cell(desc, resp)
        return SimpleNamespace(kind=TABLE, E=E, g=g, w=w)
    if desc.kind == COUNT:
        # count estimator: mean m = L Q E counts, variance s^2 = v0 + v1 m +
        # v2 m^2 > m, negative binomial with r = m^2 / (s^2 - m)
        L, v0, v1, v2 = resp
        m = L * np.asarray(desc.quench, np.float64) * E
        s2 = v0 + v1 * m + v2 * m * m
        if np.any(m <= 0) or np.any(s2 <= m):
            raise DomainError("count mean <= 0 or variance <= mean")
        return SimpleNamespace(kind=COUNT, E=E, m=m, s2=s2, r=m * m / (s2 - m))
    if desc.kind == GAUSS:
        a, b = resp
        var = a * E + b * E * E
        if np.any(var < 0):
            raise DomainError("sigma^2 < 0")
        return SimpleNamespace(kind=GAUSS, E=E, m=E.copy(), sigma=np.sqrt(var))
    L, v0, v1, v2 = resp
    p = float(desc.gg_p)
    m = L * np.asarray(desc.quench, np.float64) * E
    s2 = v0 + v1 * m + v2 * m * m
    if np.any(m <= 0) or np.any(s2 <= 0):
        raise DomainError("GG mean or variance not positive")
    tau = np.log1p(s2 / (m * m))
    k = gg_solve_shape(tau, p)
    a = m * np.exp(special.gammaln(k) - special.gammaln(k + 1.0 / p))
    return SimpleNamespace(kind=GG, E=E, m=m, s2=s2, tau=tau, k=k, a=a, p=p)


# ---------------------------------------------------------------------------
# CDF at the reco edges and the cells (Eq. 1 integrated over each reco bin).
# ---------------------------------------------------------------------------
def edge_tails(desc, cp):
    """For every column i and reco edge x_j: the smaller tail of the CDF and
    which side it is on.  lower[i, j] = True means tail = F(x_j) (<= 1/2),
    else tail = 1 - F(x_j).  F(x) = P(X < x); a zero-width Gaussian puts all
    of its mass in the reco bin [x_j, x_j+1) holding the mean."""
    x = np.asarray(desc.reco_edges, np.float64)[None, :]
    if cp.kind == GAUSS:
        m = cp.m[:, None]
        s = cp.sigma[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            z = (x - m) / s
        pos = s > 0
        lower = np.where(pos, z <= 0, x <= m)
        tail = np.where(pos, special.ndtr(np.where(lower, z, -z)), 0.0)
        return tail, lower
    k = cp.k[:, None]
    a = cp.a[:, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        y = np.where(x > 0, (np.maximum(x, 0.0) / a) ** cp.p, 0.0)
    P = special.gammainc(k, y)
    Q = special.gammaincc(k, y)
    lower = P <= 0.5
    return np.where(lower, P, Q), lower


def cells_from_tails(tail, lower):
    """R[j, i] from the edge tails: the difference is taken on the side where
    both edge values are small; a cell straddling the median is
    1 - F(x_j) - (1 - F(x_j+1))."""
    tl, th = tail[:, :-1], tail[:, 1:]
    ll, lh = lower[:, :-1], lower[:, 1:]
    cells = np.where(ll & lh, th - tl, np.where(~ll & ~lh, tl - th, 1.0 - tl - th))
    return cells.T.copy()


def response_matrix(desc, cp):
    """Dense response matrix R [N, T] (Eq. 1 on the true x reco grid).
    Tabulated response: the linear interpolation (1 - w) R_g + w R_g+1 of the
    supplied matrices (the Monte Carlo alternative to Eq. 1's analytic R)."""
    if cp.kind == TABLE:
        Rt = np.asarray(desc.table_R, np.float64)
        if Rt.shape[0] == 1:
            return Rt[0].copy()
        return (1.0 - cp.w) * Rt[cp.g] + cp.w * Rt[cp.g + 1]
    if cp.kind == COUNT:  # reco bin j is the single count n_j = x_j
        n = np.asarray(desc.reco_edges, np.float64)[:-1]
        return stats.nbinom.pmf(n[:, None], cp.r[None, :], (cp.r / (cp.r + cp.m))[None, :])
    tail, lower = edge_tails(desc, cp)
    return cells_from_tails(tail, lower)


def _gg_dF_dk(desc, cp):
    """dF(x_j)/dk_i at fixed scale a_i, by Richardson-extrapolated central
    differences of the regularized incomplete gamma in its first argument."""
    lower = edge_tails(desc, cp)[1]
    sign = np.where(lower, 1.0, -1.0)

    def side_tail(kk):
        x = np.asarray(desc.reco_edges, np.float64)[None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            y = np.where(x > 0, (np.maximum(x, 0.0) / cp.a[:, None]) ** cp.p, 0.0)
        kk = kk[:, None]
        return np.where(lower, special.gammainc(kk, y), special.gammaincc(kk, y))

    h = 1e-3 * cp.k
    d1 = (side_tail(cp.k + h) - side_tail(cp.k - h)) / (2 * h)[:, None]
    d2 = (side_tail(cp.k + h / 2) - side_tail(cp.k - h / 2)) / h[:, None]
    return sign * (4.0 * d2 - d1) / 3.0


def response_derivs(desc, cp):
    """dR/d(rho_q) [N, T] for every response parameter rho_q.

    Gaussian: dR/dsigma = -[z phi(z)]_{x_j}^{x_j+1} / sigma, with
    dsigma/da = E/(2 sigma), dsigma/db = E^2/(2 sigma).
    Generalized gamma: dR/da = -(p/a)[g(y)]_{x_j}^{x_j+1} with
    g(y) = y^k e^-y / Gamma(k); dR/dk by Richardson differences; chained
    through k(tau), tau = ln(1 + s^2/m^2), a = m Gamma(k)/Gamma(k+1/p).
    """
    x = np.asarray(desc.reco_edges, np.float64)[None, :]
    if cp.kind == GAUSS:
        s = cp.sigma[:, None]
        if np.any(cp.sigma == 0):
            raise DomainError("sigma = 0: response derivative undefined")
        z = (x - cp.m[:, None]) / s
        zphi = z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)
        dR_dsig = (-(zphi[:, 1:] - zphi[:, :-1]) / s).T      # [N, T]
        E = cp.E
        return [dR_dsig * (E / (2 * cp.sigma))[None, :],
                dR_dsig * (E * E / (2 * cp.sigma))[None, :]]
    p, k, a, m, s2 = cp.p, cp.k, cp.a, cp.m, cp.s2
    with np.errstate(divide="ignore", invalid="ignore"):
        y = np.where(x > 0, (np.maximum(x, 0.0) / a[:, None]) ** p, 0.0)
        g = np.where(y > 0, np.exp(k[:, None] * np.log(y) - y - special.gammaln(k)[:, None]), 0.0)
    dF_da = -(p / a)[:, None] * g
    dR_da = (dF_da[:, 1:] - dF_da[:, :-1]).T
    dF_dk = _gg_dF_dk(desc, cp)
    dR_dk = (dF_dk[:, 1:] - dF_dk[:, :-1]).T
    dG = special.digamma(k) + special.digamma(k + 2 / p) - 2 * special.digamma(k + 1 / p)
    dlnA_dk = special.digamma(k) - special.digamma(k + 1 / p)
    return SimpleNamespace(dR_dk=dR_dk, dR_da=dR_da, dG=dG, dlnA_dk=dlnA_dk)


def _gg_chain(cp, resp, parts):
    """Combine dR/dk and dR/da into dR/d(L, v0, v1, v2)."""
    L, v0, v1, v2 = resp
    m, s2, k, a = cp.m, cp.s2, cp.k, cp.a
    out = []
    for q in range(4):
        dm = m / L if q == 0 else np.zeros_like(m)
        ds2 = [np.zeros_like(m), np.ones_like(m), m, m * m][q] + (v1 + 2 * v2 * m) * dm
        dtau = (ds2 / (m * m) - 2 * s2 * dm / (m ** 3)) / (1 + s2 / (m * m))
        dk = dtau / parts.dG
        da = a * (dm / m + parts.dlnA_dk * dk)
        out.append(parts.dR_dk * dk[None, :] + parts.dR_da * da[None, :])
    return out


def count_derivs(desc, cp, resp):
    """Count estimator: dR/d(L, v0, v1, v2) from
    d ln P/dm = n/m - (n + r)/(r + m) and
    d ln P/dr = psi(n + r) - psi(r) + ln(r/(r + m)) + (m - n)/(r + m),
    with m = L Q E, s^2 = v0 + v1 m + v2 m^2, r = m^2/(s^2 - m)."""
    L, v0, v1, v2 = resp
    n = np.asarray(desc.reco_edges, np.float64)[:-1][:, None]
    m, s2, r = cp.m[None, :], cp.s2[None, :], cp.r[None, :]
    P = response_matrix(desc, cp)
    dP_dm = P * (n / m - (n + r) / (r + m))
    dP_dr = P * (special.digamma(n + r) - special.digamma(r) + np.log(r / (r + m)) + (m - n) / (r + m))
    d = s2 - m
    dm = [m / L, 0 * m, 0 * m, 0 * m]
    out = []
    for q in range(4):
        ds2 = [0 * m, 1 + 0 * m, m, m * m][q] + (v1 + 2 * v2 * m) * dm[q]
        dr = (2 * m * dm[q] * d - m * m * (ds2 - dm[q])) / (d * d)
        out.append(dP_dm * dm[q] + dP_dr * dr)
    return out


def response_param_derivs(desc, cp, resp):
    if cp.kind == COUNT:
        return count_derivs(desc, cp, np.asarray(resp, np.float64))
    if cp.kind == TABLE:  # R is affine in lam inside a grid cell
        Rt = np.asarray(desc.table_R, np.float64)
        if Rt.shape[0] == 1:
            return []
        grid = np.asarray(desc.table_grid, np.float64)
        return [(Rt[cp.g + 1] - Rt[cp.g]) / (grid[cp.g + 1] - grid[cp.g])]
    d = response_derivs(desc, cp)
    if cp.kind == GAUSS:
        return d
    return _gg_chain(cp, np.asarray(resp, np.float64), d)


# ---------------------------------------------------------------------------
# Species contraction (Eq. 1), pile-up (Eq. 2) and the expected counts of the
# likelihood terms (Eqs. 3-4).
# ---------------------------------------------------------------------------
def normalised_spectra(desc):
    F = np.asarray(desc.spectra, np.float64)
    return np.array([row / math.fsum(row) for row in F])


def contraction(desc, R):
    """M[j, s] = exposure * sum_i R[j, i] F[s, i]."""
    return float(desc.exposure) * (R @ normalised_spectra(desc).T)


def _pileup_conv(desc, M):
    """g_hat * M[:, s] per column, g_hat = g / sum g, a causal convolution
    truncated at the top of the reco range."""
    g = np.asarray(desc.pu_g, np.float64)
    ghat = g / math.fsum(g)
    N = M.shape[0]
    return np.stack([np.convolve(M[:, s], ghat)[:N] for s in range(M.shape[1])], axis=1)


def pileup(desc, M, p=None):
    """M'[:, s] = (1 - p) M[:, s] + p (g_hat * M[:, s]) (Eq. 2 as a mixture
    with the random-trigger spectrum); p defaults to the model's fixed
    fraction."""
    p = float(desc.pu_frac) if p is None else float(p)
    if p == 0.0 or desc.pu_g is None:
        return M.copy()
    return (1.0 - p) * M + p * _pileup_conv(desc, M)


def pileup_dp(desc, M):
    """dM'/dp = g_hat * M - M: M' is affine in the pile-up fraction."""
    if desc.pu_g is None:
        return np.zeros_like(M)
    return _pileup_conv(desc, M) - M


def expected(desc, Mp, r):
    """Expected counts per likelihood term, linear in both M' and r.

    Single histogram: mu = M' r.
    Multivariate (Eq. 4): with c_sub = (1 - t) r, c_tag = t r:
      vetoed mu_sub = M' c_sub, tagged mu_tag = M' c_tag (Eq. 3);
      radial nu_k = sum_s c_sub,s (sum_{j in radial window} M'_js) rho_sk;
      pulse shape lambda_jk = sum_s M'_js c_sub,s T_sk (rows of the fit
      window), all built from the TFC-vetoed expectation.
    Joint (the alternative to the additive terms): the vetoed events in one
    energy x radius x pulse-shape histogram with lambda_jkl = sum_s M'_js
    c_sub,s rho_sk T_sl, plus the tagged term."""
    r = np.asarray(r, np.float64)
    j0, j1 = desc.win
    if not desc.multivariate:
        return {"energy": (Mp @ r)[j0:j1]}
    t = np.asarray(desc.tag_frac, np.float64)
    c_sub = (1.0 - t) * r
    c_tag = t * r
    if getattr(desc, "joint", False):
        # joint energy x radius x pulse-shape PDF of the vetoed events instead
        # of three additive terms: lambda_jkl = sum_s M'_js c_sub,s rho_sk T_sl
        rho = np.asarray(desc.rad_tmpl, np.float64)
        T = np.asarray(desc.ps_tmpl, np.float64)
        lam = np.einsum("js,sk,sl->jkl", Mp[j0:j1] * c_sub[None, :], rho, T)
        return {"joint": lam, "tagged": (Mp @ c_tag)[j0:j1]}
    out = {"energy": (Mp @ c_sub)[j0:j1], "tagged": (Mp @ c_tag)[j0:j1]}
    if desc.rad_tmpl is not None:
        rw0, rw1 = desc.rad_win
        A = c_sub * Mp[rw0:rw1].sum(axis=0)
        out["radial"] = A @ np.asarray(desc.rad_tmpl, np.float64)
    if desc.ps_tmpl is not None:
        out["ps"] = ((Mp * c_sub[None, :]) @ np.asarray(desc.ps_tmpl, np.float64))[j0:j1]
    return out


def observed(desc, data):
    j0, j1 = desc.win
    if getattr(desc, "joint", False):
        return {"joint": np.asarray(data.joint, np.float64)[j0:j1],
                "tagged": np.asarray(data.tagged, np.float64)[j0:j1]}
    out = {"energy": np.asarray(data.energy, np.float64)[j0:j1]}
    if desc.multivariate:
        out["tagged"] = np.asarray(data.tagged, np.float64)[j0:j1]
        if desc.rad_tmpl is not None:
            out["radial"] = np.asarray(data.radial, np.float64)
        if desc.ps_tmpl is not None:
            out["ps"] = np.asarray(data.ps, np.float64)[j0:j1]
    return out


# ---------------------------------------------------------------------------
# Binned Poisson NLL without the data-only constant: sum (mu - n ln mu).
# ---------------------------------------------------------------------------
def nll_terms(mu, n):
    mu = np.asarray(mu, np.float64).ravel()
    n = np.asarray(n, np.float64).ravel()
    if not np.all(np.isfinite(mu)) or np.any(mu < 0) or np.any((mu == 0) & (n > 0)):
        raise DomainError("expected count negative, or zero where counts > 0")
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(n > 0, mu - n * np.log(mu), mu)


def split_theta(desc, theta):
    theta = np.asarray(theta, np.float64)
    if theta.shape != (desc.P,):
        raise ValueError(f"theta must have {desc.P} entries")
    if not np.all(np.isfinite(theta)):
        raise DomainError("non-finite theta")
    return theta[: desc.S], theta[desc.S: desc.S + desc.n_resp]


def pu_fraction(desc, theta):
    """The pile-up fraction: the last parameter when it is floated (it must
    lie in [0, 1]), else the model's fixed value."""
    if not getattr(desc, "pu_float", False):
        return float(desc.pu_frac)
    p = float(np.asarray(theta, np.float64)[-1])
    if not (0.0 <= p <= 1.0):
        raise DomainError("pile-up fraction outside [0, 1]")
    return p


def forward(desc, theta):
    r, resp = split_theta(desc, theta)
    p = pu_fraction(desc, theta)
    cp = column_params(desc, resp)
    R = response_matrix(desc, cp)
    M = contraction(desc, R)
    Mp = pileup(desc, M, p)
    return SimpleNamespace(cp=cp, R=R, M=M, Mp=Mp, r=r, resp=resp, p=p, mu=expected(desc, Mp, r))


def nll(desc, data, theta):
    """Extended binned Poisson NLL (all terms of Eq. 3 / Eq. 4)."""
    f = forward(desc, theta)
    obs = observed(desc, data)
    return math.fsum(math.fsum(nll_terms(f.mu[key], obs[key])) for key in f.mu)


def lnfact(desc, data):
    """Sum of ln Gamma(n + 1) over all bins entering the NLL."""
    obs = observed(desc, data)
    return math.fsum(math.fsum(special.gammaln(v.ravel() + 1.0)) for v in obs.values())


def grad(desc, data, theta):
    """Gradient of the NLL, forward mode: for every parameter q the
    derivatives of the expected counts dmu/dq are formed explicitly and
    contracted with w = 1 - n/mu."""
    return nll_grad(desc, data, theta)[1]


def nll_grad(desc, data, theta):
    f = forward(desc, theta)
    obs = observed(desc, data)
    val = math.fsum(math.fsum(nll_terms(f.mu[key], obs[key])) for key in f.mu)
    w = {}
    for key in f.mu:
        mu = f.mu[key]
        n = obs[key]
        with np.errstate(divide="ignore", invalid="ignore"):
            w[key] = np.where(n > 0, 1.0 - n / mu, 1.0)

    def contract(dmu):
        return math.fsum(math.fsum((w[key] * dmu[key]).ravel()) for key in w)

    g = np.zeros(desc.P)
    for s in range(desc.S):
        e = np.zeros(desc.S)
        e[s] = 1.0
        g[s] = contract(expected(desc, f.Mp, e))
    for q, dR in enumerate(response_param_derivs(desc, f.cp, f.resp)):
        dMp = pileup(desc, contraction(desc, dR), f.p)
        g[desc.S + q] = contract(expected(desc, dMp, f.r))
    if getattr(desc, "pu_float", False):
        g[desc.P - 1] = contract(expected(desc, pileup_dp(desc, f.M), f.r))
    return val, g


def per_species_expected(desc, theta):
    """M' [N, S]: expected counts per unit rate of every species, after the
    response and pile-up, at the response parameters of theta."""
    return forward(desc, theta).Mp


def support_edges(desc, theta, q=1e-12):
    """CDF evaluations one response sweep needs (Eq. 1 integrated over the
    reco bins): for every column, the reco edges whose CDF lies in [q, 1 - q]
    plus the edge just outside on each side, which closes the first and last
    cell of the column's support."""
    _, resp = split_theta(desc, theta)
    tail, _ = edge_tails(desc, column_params(desc, resp))
    n_edges = tail.shape[1]
    total = 0
    for row in tail >= q:
        idx = np.flatnonzero(row)
        if idx.size:
            total += int(min(idx[-1] + 1, n_edges - 1) - max(idx[0] - 1, 0) + 1)
    return total


def support_cells(desc, theta, q=1e-12):
    """Cells one response sweep needs (Eq. 1 integrated over the reco bins):
    for every column, the cells between the edges that support_edges counts
    (one fewer than its edges; none for a column without support)."""
    _, resp = split_theta(desc, theta)
    tail, _ = edge_tails(desc, column_params(desc, resp))
    n_edges = tail.shape[1]
    total = 0
    for row in tail >= q:
        idx = np.flatnonzero(row)
        if idx.size:
            total += int(min(idx[-1] + 1, n_edges - 1) - max(idx[0] - 1, 0))
    return total


def _scale(desc, data, theta, weight):
    """sum over bins of weight_b |dmu_b/dq| for every parameter q."""
    f = forward(desc, theta)
    obs = observed(desc, data)
    a = {}
    for key in f.mu:
        with np.errstate(divide="ignore", invalid="ignore"):
            a[key] = weight(f.mu[key], obs[key])

    def contract(dmu):
        return math.fsum(math.fsum((a[key] * np.abs(dmu[key])).ravel()) for key in a)

    sc = np.zeros(desc.P)
    for s in range(desc.S):
        e = np.zeros(desc.S)
        e[s] = 1.0
        sc[s] = contract(expected(desc, f.Mp, e))
    for q, dR in enumerate(response_param_derivs(desc, f.cp, f.resp)):
        dMp = pileup(desc, contraction(desc, dR), f.p)
        sc[desc.S + q] = contract(expected(desc, dMp, f.r))
    if getattr(desc, "pu_float", False):
        sc[desc.P - 1] = contract(expected(desc, pileup_dp(desc, f.M), f.r))
    return sc


def grad_scale(desc, data, theta):
    """Magnitude scale of each gradient component q: the sum over bins of the
    absolute summands of dNLL/dq = sum_b (1 - n_b/mu_b) dmu_b/dq, that is
    sum_b |1 - n_b/mu_b| |dmu_b/dq| (a bin with n_b = 0 has weight 1).
    Gradient tolerances are relative to it, because the gradient itself goes
    to zero at the minimum."""
    return _scale(desc, data, theta, lambda mu, n: np.where(n > 0, np.abs(1.0 - n / mu), 1.0))


def grad_scale_abs(desc, data, theta):
    """A looser scale, reported beside grad_scale: sum over bins of
    |dmu_b/dq| (1 + n_b/mu_b), the size of the two terms that cancel in each
    summand (1 - n_b/mu_b) dmu_b/dq.  Near the minimum it is roughly
    2 sum_b |dmu_b/dq|, one to two orders above grad_scale."""
    return _scale(desc, data, theta, lambda mu, n: np.where(n > 0, 1.0 + n / mu, 1.0))
