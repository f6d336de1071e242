"""FP64 CPU oracle for the F-chi2 period search.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this module: only the test suite, the smoke check of the entry module
and the CPU-baseline leg of the benchmark use it.  It shares no code, tables or
helpers with the HIP library.

What it computes is the plain definition of the method (Palmer, "A Fast
Chi-squared Technique For Period Search of Irregularly Sampled Data",
Sections 2 and 3c-3e), evaluated directly at every requested frequency:

* the model is the Fourier series truncated at H harmonics (eq. eqtrunc) with
  basis M_0 = 1, M_{2h-1} = sin(2 pi h f t), M_{2h} = cos(2 pi h f t)
  (Section 2, the component functions following the linear/non-linear split);
* chi2(P) = sum_i (M(P, t_i) - x_i)^2 / sigma_i^2 (eq. eqchigen);
* the normal equations alpha_jk = sum_i M_j M_k / sigma_i^2 and
  beta_j = sum_i M_j x_i / sigma_i^2 (Section 2), built here from the centred
  data y = x - xbar with xbar the weighted mean (Section 3b), so beta_0 = 0;
* chi2_min = X - beta^T alpha^{-1} beta (eq. eqchix), hence the reduction
  Delta chi2 = chi2_0 - chi2_min = beta^T alpha^{-1} beta with
  chi2_0 = sum_i (x_i - xbar)^2 / sigma_i^2 (Section 3d);
* coefficients A = alpha^{-1} beta (eq. eqcoeffs), with xbar added back to A_0
  (Section 3b).

Every H' = 1..H is solved from its own leading (2H'+1) block of alpha (the
basis is ordered so that the H' model is a prefix of the H model).  Phases are
taken as 2 pi * frac(h f (t - T0)) from the FP64 product, with no angle
addition recurrences; T0 = min t (Section 3b allows any T0 <= all t_i; the
fit is invariant under a time shift).

Readings of points where the paper is silent (documented with the design):
* the f = 0 bin has a singular alpha (sin columns vanish, cos columns repeat
  the constant); its Delta chi2 is defined as 0 and it is flagged;
* a block whose Cholesky factorisation fails, or whose diagonally scaled
  condition number exceeds 1e12, is solved with a pseudo-inverse
  (rcond 1e-12) and flagged;
* the gradient is the closed form that follows from eq. eqchigen and eq.
  eqchix by the envelope theorem:
      d Delta / d x_i     = 2 w_i yhat_i
      d Delta / d sigma_i = -(2 w_i / sigma_i) yhat_i (2 y_i - yhat_i)
  where w = sigma^-2, y = x - xbar and yhat is the fitted (centred) model.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

FLAG_PINV = 1      # Cholesky failed or the block was too ill-conditioned
FLAG_LOW_F = 2     # f < 1 / span: variability rather than periodicity
FLAG_DC = 4        # the f = 0 bin

KAPPA_PINV = 1e12  # scaled condition number above which the pinv is used


def moments(t, x, sigma):
    """Weights, weighted mean and the null chi2 (Section 3b and 3d)."""
    t = np.asarray(t, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    w = 1.0 / (sigma * sigma)
    W = np.sum(w)
    xbar = np.sum(w * x) / W
    y = x - xbar
    chi2_0 = np.sum(w * y * y)
    T0 = np.min(t)
    span = np.max(t) - T0
    return dict(w=w, W=W, xbar=xbar, y=y, chi2_0=chi2_0, T0=T0, span=span)


def basis(tau, f, H):
    """Design matrix [n, 2H+1]: columns 1, sin h, cos h for h = 1..H.

    The phase of harmonic h is 2 pi frac(h f tau), evaluated directly in FP64.
    """
    tau = np.asarray(tau, dtype=np.float64)
    n = tau.shape[0]
    M = np.empty((n, 2 * H + 1), dtype=np.float64)
    M[:, 0] = 1.0
    for h in range(1, H + 1):
        cyc = (h * f) * tau
        theta = 2.0 * np.pi * (cyc - np.floor(cyc))
        M[:, 2 * h - 1] = np.sin(theta)
        M[:, 2 * h] = np.cos(theta)
    return M


def normal_equations(tau, w, y, f, H):
    """alpha = sum_i w_i M M^T, beta = sum_i w_i y_i M (Section 2)."""
    M = basis(tau, f, H)
    alpha = M.T @ (w[:, None] * M)
    beta = M.T @ (w * y)
    return alpha, beta, M


def scaled_condition(alpha):
    """Condition number of D^-1/2 alpha D^-1/2 with D = diag(alpha)."""
    d = np.sqrt(np.diag(alpha))
    if np.any(d <= 0) or not np.all(np.isfinite(d)):
        return np.inf
    s = alpha / np.outer(d, d)
    return np.linalg.cond(s)


def _solve_block(a, b):
    """Return (A, flagged) with A = a^-1 b, Cholesky first, pinv on failure."""
    kap = scaled_condition(a)
    if np.isfinite(kap) and kap <= KAPPA_PINV:
        try:
            c = scipy.linalg.cho_factor(a, lower=True, check_finite=True)
            return scipy.linalg.cho_solve(c, b), False
        except np.linalg.LinAlgError:
            pass
    return np.linalg.pinv(a, rcond=1e-12, hermitian=True) @ b, True


def dchi2(t, x, sigma, freqs, H, *, with_coeffs=False):
    """Delta chi2(f, H') for every f in `freqs` and H' = 1..H.

    Returns a dict with
      dchi2  [H, nf]  Delta chi2 for H' = 1..H (row H'-1)
      kappa  [nf]     scaled condition number of the full (2H+1) alpha
      flags  [nf]     FLAG_* bits
      coeffs [nf, 2H+1] (if with_coeffs) coefficients of the H model, xbar
                      added back to A_0, in the basis of absolute time t - T0
      chi2_0, xbar, W, T0, span
    """
    m = moments(t, x, sigma)
    tau = np.asarray(t, dtype=np.float64) - m["T0"]
    freqs = np.asarray(freqs, dtype=np.float64)
    nf = freqs.shape[0]
    out = np.zeros((H, nf), dtype=np.float64)
    kappa = np.zeros(nf, dtype=np.float64)
    flags = np.zeros(nf, dtype=np.uint8)
    coeffs = np.zeros((nf, 2 * H + 1), dtype=np.float64) if with_coeffs else None
    for j, f in enumerate(freqs):
        if f == 0.0:
            flags[j] |= FLAG_DC
            kappa[j] = np.inf
            if with_coeffs:
                coeffs[j, 0] = m["xbar"]
            continue
        if m["span"] > 0 and f < 1.0 / m["span"]:
            flags[j] |= FLAG_LOW_F
        alpha, beta, _ = normal_equations(tau, m["w"], m["y"], f, H)
        kappa[j] = scaled_condition(alpha)
        for hp in range(1, H + 1):
            d = 2 * hp + 1
            A, bad = _solve_block(alpha[:d, :d], beta[:d])
            if bad:
                flags[j] |= FLAG_PINV
            out[hp - 1, j] = float(beta[:d] @ A)
            if with_coeffs and hp == H:
                coeffs[j, :] = A
                coeffs[j, 0] += m["xbar"]
    res = dict(dchi2=out, kappa=kappa, flags=flags, chi2_0=m["chi2_0"],
               xbar=m["xbar"], W=m["W"], T0=m["T0"], span=m["span"])
    if with_coeffs:
        res["coeffs"] = coeffs
    return res


def fitted(t, x, sigma, f, H):
    """Centred fitted model yhat_i of the H-harmonic fit at frequency f."""
    m = moments(t, x, sigma)
    tau = np.asarray(t, dtype=np.float64) - m["T0"]
    alpha, beta, M = normal_equations(tau, m["w"], m["y"], f, H)
    A, _ = _solve_block(alpha, beta)
    return M @ A, m


def grad(t, x, sigma, terms):
    """Closed-form gradient of L = sum_p g_p * Delta chi2(f_p, H'_p).

    `terms` is an iterable of (f, H', g).  Returns (dL/dx, dL/dsigma) in FP64.
    """
    x = np.asarray(x, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    gx = np.zeros_like(x)
    gs = np.zeros_like(sigma)
    for f, hp, g in terms:
        yhat, m = fitted(t, x, sigma, f, hp)
        w, y = m["w"], m["y"]
        gx += g * 2.0 * w * yhat
        gs += g * (-(2.0 * w / sigma) * yhat * (2.0 * y - yhat))
    return gx, gs


def log_chi2_sf_even(d, hp):
    """ln of the upper tail of the chi2 law with 2 hp degrees of freedom at d.

    Uses the Poisson identity: for even degrees of freedom the chi2 tail at d
    equals P(N <= hp - 1) for N Poisson with mean d/2, so
    ln Q = logsumexp_j (j ln u - u - ln j!), j < hp, u = d/2 (d < 0 -> 0).
    Unlike a log of the tail itself, this stays finite for any d.
    """
    import scipy.special
    d = np.maximum(np.asarray(d, dtype=np.float64), 0.0)
    u = 0.5 * d
    j = np.arange(hp, dtype=np.float64)
    with np.errstate(divide="ignore"):
        lu = np.log(u)
    terms = j[:, None] * np.where(u > 0, lu, 0.0)[None, :] - u[None, :] \
        - scipy.special.gammaln(j + 1.0)[:, None]
    terms[1:, u == 0] = -np.inf                 # u^j = 0 for j >= 1 at u = 0
    return scipy.special.logsumexp(terms, axis=0).reshape(np.shape(d))


def log_significance(dchi2, k, H):
    """ln p(f_k) = ln k + ln Q(Delta chi2 | 2H'), rows H' = 1..H (Section 3e).

    p(f) is the chance probability of a reduction this large at a frequency
    up to f: the bin index (trials so far) times the upper tail of the chi2
    distribution with 2H' degrees of freedom (the model's extra parameters).
    k = 0 gives ln p = -inf.
    """
    dchi2 = np.asarray(dchi2, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    out = np.empty_like(dchi2)
    with np.errstate(divide="ignore"):
        lk = np.log(k)
    for hp in range(1, dchi2.shape[0] + 1):
        out[hp - 1] = lk + log_chi2_sf_even(dchi2[hp - 1], hp)
    return out


def dchi2_adjusted(dchi2, chi2_0, n):
    """Delta chi2_adj = Delta chi2 / (chi2_best / N_dof), rows H' = 1..H (Section 3e).

    Reading of the printed denominator: chi2_best = chi2_0 - max_k Delta chi2
    is the minimum chi2 of the best fit and N_dof = n - 2H' - 1 its degrees of
    freedom, so the denominator is the best fit's reduced chi2 (the source
    noise relative to the stated errors).  The maximum is over the bins given.
    N_dof <= 0 gives NaN.
    """
    dchi2 = np.asarray(dchi2, dtype=np.float64)
    out = np.empty_like(dchi2)
    for hp in range(1, dchi2.shape[0] + 1):
        best = chi2_0 - np.max(dchi2[hp - 1])
        ndof = n - 2 * hp - 1
        out[hp - 1] = dchi2[hp - 1] * ndof / best if ndof > 0 else np.nan
    return out


def top_candidates(dchi2_row, freqs, span, hp, K, k_lo=0):
    """Best K candidate bins of one row (H' = hp) by ln p (Section 3e).

    Candidates: bins k with k >= max(k_lo, 1), f_k >= 1/span, k <= N - 2 and
    D[k] > D[k-1], D[k] >= D[k+1] (strict on the left: a plateau counts
    once).  Ranked by ln p = ln k + ln Q(D[k] | 2hp) ascending, ties to the
    lower k.  Also returns the largest D over the eligible bins (k up to
    N - 1), from which chi2_best = chi2_0 - max follows.
    Returns (idx [<=K], log_p [<=K], dmax or -inf).
    """
    d = np.asarray(dchi2_row, dtype=np.float64)
    freqs = np.asarray(freqs, dtype=np.float64)
    n = d.shape[0]
    k = np.arange(n)
    elig = (k >= max(int(k_lo), 1))
    if span > 0:
        elig &= freqs * span >= 1.0
    dmax = float(np.max(d[elig])) if np.any(elig) else -np.inf
    cand = []
    for j in np.nonzero(elig)[0]:
        if j > n - 2:
            continue
        if d[j] > d[j - 1] and d[j] >= d[j + 1]:
            lp = np.log(j) + float(log_chi2_sf_even(np.array([d[j]]), hp)[0])
            cand.append((lp, j))
    cand.sort()
    cand = cand[:K]
    return (np.array([c[1] for c in cand], dtype=np.int64),
            np.array([c[0] for c in cand], dtype=np.float64), dmax)


def floor_gridded_times(t, df, L):
    """Times as the floor gridding of Section 3b sees them.

    Each time is replaced by the start of its cell: with T0 = min t and cell
    width 1/(df L), j = floor(((t - T0) df) L) (evaluated in this order, in
    FP64) and the returned time is T0 + j / (df L).  Running `dchi2` on these
    times gives what a floor-gridded search computes, sensitivity loss
    included.
    """
    t = np.asarray(t, dtype=np.float64)
    T0 = np.min(t)
    j = np.floor(((t - T0) * df) * float(L))
    return T0 + j / (df * float(L))


def detrend(t, x, sigma, degree):
    """Residuals of the weighted least-squares polynomial fit of x in t.

    The reference implementation of the paper can remove a polynomial trend
    (up to t^3 in its Section 4 example) before the search.  The fit minimises
    sum w (x - p(t))^2, w = sigma^-2, over polynomials of the given degree;
    it is solved here with lstsq on the monomials of u = 2 (t - T0) / span - 1
    (the same polynomial space as powers of t, better conditioned).
    """
    t = np.asarray(t, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    sw = 1.0 / np.asarray(sigma, dtype=np.float64)
    T0, span = np.min(t), np.max(t) - np.min(t)
    u = 2.0 * (t - T0) / span - 1.0 if span > 0 else np.zeros_like(t)
    V = np.stack([u ** j for j in range(degree + 1)], axis=1)
    c, *_ = np.linalg.lstsq(V * sw[:, None], x * sw, rcond=None)
    return x - V @ c


def gate_mask(res, freqs, kappa_max):
    """Bins on which parity is judged: k >= 1, f >= 1/span, kappa <= kappa_max."""
    freqs = np.asarray(freqs, dtype=np.float64)
    ok = freqs > 0.0
    if res["span"] > 0:
        ok &= freqs >= 1.0 / res["span"]
    ok &= res["kappa"] <= kappa_max
    return ok


def rel_err(d_gpu, d_ora):
    """|d_gpu - d_ora| / max(d_ora, 2H') with rows indexed by H' - 1.

    The floor 2H' is the mean of Delta chi2 under the null hypothesis
    (Section 3e: 2H additional free parameters).
    """
    d_gpu = np.asarray(d_gpu, dtype=np.float64)
    d_ora = np.asarray(d_ora, dtype=np.float64)
    H = d_ora.shape[0]
    floor = (2.0 * np.arange(1, H + 1, dtype=np.float64))[:, None]
    return np.abs(d_gpu - d_ora) / np.maximum(d_ora, floor)
