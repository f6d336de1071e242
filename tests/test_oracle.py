"""Pins for the FP64 oracle against facts fixed outside it.

Each test checks the oracle against something other than itself: a different
least-squares route (SVD via lstsq on the design matrix of eq. eqtrunc), a
textbook closed form (the classical periodogram on an equally spaced grid),
invariances of the chi2 fit (Section 2), exact recovery of a noiseless signal,
the null distribution of Delta chi2 (Section 2 and 3e: chi2 with 2H degrees of
freedom), the printed H = 2 normal matrix of Section 3c, and finite
differences for the closed-form gradient.
"""
import math
import os

import numpy as np
import pytest
import scipy.stats

from oracle import fchi2_oracle as ora

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_curve(rng, n, span=50.0, offset=0.0):
    t = np.sort(rng.uniform(0.0, span, n)) + offset
    s = rng.uniform(0.05, 0.3, n)
    x = 0.3 * np.sin(2 * np.pi * t / 3.1) + s * rng.standard_normal(n)
    return t, x, s


def _lstsq_dchi2(t, x, s, f, H):
    """Delta chi2 by brute force: two weighted lstsq fits on absolute t."""
    sw = 1.0 / s
    cols = [np.ones_like(t)]
    for h in range(1, H + 1):
        cols.append(np.sin(2 * np.pi * h * f * t))
        cols.append(np.cos(2 * np.pi * h * f * t))
    M = np.stack(cols, axis=1)
    A, *_ = np.linalg.lstsq(M * sw[:, None], x * sw, rcond=None)
    chi2 = np.sum(((M @ A - x) * sw) ** 2)
    c, *_ = np.linalg.lstsq(sw[:, None], x * sw, rcond=None)
    chi2_0 = np.sum(((c[0] - x) * sw) ** 2)
    return chi2_0 - chi2, A


@pytest.mark.parametrize("seed", range(6))
def test_matches_bruteforce_lstsq(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(12, 64))
    H = int(rng.integers(1, 5))
    t, x, s = _rand_curve(rng, n)
    freqs = rng.uniform(0.05, 3.0, 12)
    res = ora.dchi2(t, x, s, freqs, H, with_coeffs=True)
    for j, f in enumerate(freqs):
        for hp in range(1, H + 1):
            if n < 2 * hp + 1 + 2:
                continue
            ref, A = _lstsq_dchi2(t, x, s, f, hp)
            got = res["dchi2"][hp - 1, j]
            assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref)), (f, hp, got, ref)


def test_coefficients_match_lstsq_absolute_time():
    """A from eq. eqcoeffs, with xbar added back to A_0 (Section 3b)."""
    rng = np.random.default_rng(7)
    t, x, s = _rand_curve(rng, 40)
    t = t - t.min()            # oracle coefficients are in tau = t - T0
    f, H = 0.37, 3
    res = ora.dchi2(t, x, s, [f], H, with_coeffs=True)
    _, A = _lstsq_dchi2(t, x, s, f, H)
    np.testing.assert_allclose(res["coeffs"][0], A, rtol=1e-9, atol=1e-11)


def test_periodogram_closed_form():
    """Equal spacing, equal errors, f = k/n with 2Hk < n: orthogonal basis.

    Then Delta(H') = (2 w / n) sum_{h <= H'} |DFT(y)[h k]|^2, the classical
    periodogram summed over harmonics.
    """
    rng = np.random.default_rng(11)
    n, H = 256, 4
    t = np.arange(n, dtype=np.float64)
    s = np.full(n, 0.2)
    x = rng.standard_normal(n) * 0.2 + 0.1 * np.cos(2 * np.pi * 5 * t / n)
    ks = [1, 3, 5, 17, 31]
    freqs = np.array(ks, dtype=np.float64) / n
    res = ora.dchi2(t, x, s, freqs, H)
    y = x - x.mean()
    F = np.fft.fft(y)
    w = 1.0 / 0.2 ** 2
    for j, k in enumerate(ks):
        acc = 0.0
        for hp in range(1, H + 1):
            acc += (2.0 * w / n) * abs(F[hp * k]) ** 2
            np.testing.assert_allclose(res["dchi2"][hp - 1, j], acc, rtol=1e-10)


def test_invariants():
    rng = np.random.default_rng(21)
    t, x, s = _rand_curve(rng, 60)
    H = 3
    freqs = np.linspace(0.05, 2.0, 25)
    base = ora.dchi2(t, x, s, freqs, H)
    d = base["dchi2"]
    assert np.all(d >= -1e-9)
    assert np.all(np.diff(d, axis=0) >= -1e-9)           # nondecreasing in H'
    assert np.all(d <= base["chi2_0"] * (1 + 1e-12))      # bounded by chi2_0

    for c in (0.37, 2.45e6):                              # time shift
        sh = ora.dchi2(t + c, x, s, freqs, H)["dchi2"]
        np.testing.assert_allclose(sh, d, rtol=1e-7, atol=1e-9)

    a, b = -2.5, 7.0                                      # affine in x
    af = ora.dchi2(t, a * x + b, abs(a) * s, freqs, H)["dchi2"]
    np.testing.assert_allclose(af, d, rtol=1e-10, atol=1e-12)

    sc = ora.dchi2(t, x, 3.0 * s, freqs, H)["dchi2"]      # sigma -> c sigma
    np.testing.assert_allclose(sc, d / 9.0, rtol=1e-10, atol=1e-12)

    p = rng.permutation(t.shape[0])                       # permutation
    pm = ora.dchi2(t[p], x[p], s[p], freqs, H)["dchi2"]
    np.testing.assert_allclose(pm, d, rtol=1e-10, atol=1e-12)

    tt = np.concatenate([t, t])                           # duplicate, sigma*sqrt2
    dup = ora.dchi2(tt, np.concatenate([x, x]),
                    np.concatenate([s, s]) * np.sqrt(2.0), freqs, H)["dchi2"]
    np.testing.assert_allclose(dup, d, rtol=1e-10, atol=1e-12)


def test_exact_recovery_noiseless():
    """A noiseless H_sig-harmonic signal at f0 is fitted exactly for H' >= H_sig."""
    rng = np.random.default_rng(31)
    n = 80
    t = np.sort(rng.uniform(0.0, 40.0, n))
    s = rng.uniform(0.1, 0.3, n)
    f0, Hs = 0.731, 2
    A_true = np.array([1.5, 0.4, -0.2, 0.1, 0.25])  # const, s1, c1, s2, c2
    tau = t - t.min()
    x = A_true[0] + sum(A_true[2 * h - 1] * np.sin(2 * np.pi * h * f0 * tau)
                        + A_true[2 * h] * np.cos(2 * np.pi * h * f0 * tau)
                        for h in range(1, Hs + 1))
    res = ora.dchi2(t, x, s, [f0], 3, with_coeffs=True)
    chi2_0 = res["chi2_0"]
    assert res["dchi2"][0, 0] < chi2_0 * (1 - 1e-3)
    np.testing.assert_allclose(res["dchi2"][1:, 0], chi2_0, rtol=1e-10)
    np.testing.assert_allclose(res["coeffs"][0, :5], A_true, atol=1e-9)
    np.testing.assert_allclose(res["coeffs"][0, 5:], 0.0, atol=1e-9)


@pytest.mark.parametrize("hp", [1, 3])
def test_null_distribution_is_chi2_2H(hp):
    """Pure Gaussian noise: Delta(f, H') ~ chi2 with 2H' dof (Sections 2, 3e)."""
    rng = np.random.default_rng(41 + hp)
    n, trials = 40, 1500
    t = np.sort(rng.uniform(0.0, 30.0, n))
    s = rng.uniform(0.05, 0.3, n)
    f = 0.4137
    vals = np.empty(trials)
    for k in range(trials):
        x = 3.0 + s * rng.standard_normal(n)
        vals[k] = ora.dchi2(t, x, s, [f], hp)["dchi2"][hp - 1, 0]
    stat = scipy.stats.kstest(vals, scipy.stats.chi2(2 * hp).cdf)
    assert stat.pvalue > 1e-3, stat
    # A 1/sigma (instead of 1/sigma^2) weight would scale the mean badly.
    assert abs(vals.mean() / (2 * hp) - 1.0) < 0.1


def _parse_terms(expr, Q, P):
    total = 0.0
    for tok in expr.split():
        coef, sym = tok.split("*")
        val = {"Qr": lambda n: Q[n].real, "Qi": lambda n: Q[n].imag,
               "Pr": lambda n: P[n].real, "Pi": lambda n: P[n].imag}[sym[:2]](int(sym[2:]))
        total += float(coef) * val
    return total


def test_h2_printed_normal_matrix():
    """Section 3c's H = 2 alpha/beta, with the sign reading of its fixture."""
    rng = np.random.default_rng(51)
    t, x, s = _rand_curve(rng, 50)
    f = 0.613
    m = ora.moments(t, x, s)
    tau = t - m["T0"]
    Q = [np.sum(m["w"] * np.exp(2j * np.pi * n * f * tau)) for n in range(5)]
    P = [np.sum(m["w"] * m["y"] * np.exp(2j * np.pi * n * f * tau)) for n in range(3)]
    alpha, beta, _ = ora.normal_equations(tau, m["w"], m["y"], f, 2)
    printed = np.zeros((5, 5))
    reading = np.zeros((5, 5))
    b_read = np.zeros(5)
    with open(os.path.join(GOLDEN, "h2_normal_matrix.txt")) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            kind, r, c, rest = line.split(maxsplit=3)
            pr, rd = rest.split("|")
            if kind == "alpha":
                printed[int(r), int(c)] = 0.5 * _parse_terms(pr, Q, P)
                reading[int(r), int(c)] = 0.5 * _parse_terms(rd, Q, P)
            else:
                b_read[int(r)] = _parse_terms(rd, Q, P)
    scale = np.max(np.abs(alpha))
    assert np.max(np.abs(reading - alpha)) <= 1e-12 * scale
    assert np.max(np.abs(b_read - beta)) <= 1e-12 * np.max(np.abs(beta))
    # The printed matrix is off by exactly +-Qi_1 at the four named entries.
    diff = printed - alpha
    mask = np.zeros((5, 5), dtype=bool)
    for r, c in [(1, 4), (4, 1), (2, 3), (3, 2)]:
        mask[r, c] = True
        assert abs(abs(diff[r, c]) - abs(Q[1].imag)) <= 1e-10 * scale
    assert np.max(np.abs(diff[~mask])) <= 1e-12 * scale


def test_gradient_closed_form_vs_finite_differences():
    rng = np.random.default_rng(61)
    t, x, s = _rand_curve(rng, 30)
    terms = [(0.52, 2, 1.0), (1.37, 3, 0.5)]
    gx, gs = ora.grad(t, x, s, terms)

    def loss(xx, ss):
        tot = 0.0
        for f, hp, g in terms:
            tot += g * ora.dchi2(t, xx, ss, [f], hp)["dchi2"][hp - 1, 0]
        return tot

    for i in (0, 7, 19, 29):
        h = 1e-3
        e = np.zeros_like(x)
        e[i] = h
        fd = (loss(x + e, s) - loss(x - e, s)) / (2 * h)
        assert abs(fd - gx[i]) <= 1e-7 * max(1.0, abs(gx[i])), (i, fd, gx[i])
        h = 1e-4 * s[i]
        e = np.zeros_like(s)
        e[i] = h
        fd = (loss(x, s + e) - loss(x, s - e)) / (2 * h)
        assert abs(fd - gs[i]) <= 1e-5 * max(1.0, abs(gs[i])), (i, fd, gs[i])


def test_dc_bin_and_flags():
    rng = np.random.default_rng(71)
    t, x, s = _rand_curve(rng, 30)
    res = ora.dchi2(t, x, s, [0.0, 0.001, 0.5], 2)
    assert res["dchi2"][0, 0] == 0.0 and res["flags"][0] & ora.FLAG_DC
    assert res["flags"][1] & ora.FLAG_LOW_F
    assert not res["flags"][2] & (ora.FLAG_LOW_F | ora.FLAG_DC)


def test_rel_err_floor():
    d_ora = np.array([[0.5, 10.0], [1.0, 20.0]])
    d_gpu = d_ora + 0.01
    e = ora.rel_err(d_gpu, d_ora)
    np.testing.assert_allclose(e, [[0.01 / 2, 0.01 / 10], [0.01 / 4, 0.01 / 20]])


def test_log_significance_even_dof_closed_form():
    """Upper chi2 tail with 2H dof: exp(-x/2) sum_{j<H} (x/2)^j / j!, and scipy's
    chi2.logsf where that does not underflow."""
    x = np.array([[0.0, 0.5, 3.0, 40.0, 700.0, 1400.0, 3e4, 2e6]] * 8)
    k = np.array([1, 2, 10, 1000, 7, 3, 123456, 5])
    got = ora.log_significance(x, k, 8)
    for hp in range(1, 9):
        for j in range(x.shape[1]):
            xx = x[hp - 1, j]
            s = sum((xx / 2) ** i / math.factorial(i) for i in range(hp))
            ref = math.log(k[j]) - xx / 2 + math.log(s)
            assert abs(got[hp - 1, j] - ref) <= 1e-12 * max(1.0, abs(ref)), (hp, xx)
            if xx <= 1400.0:
                sp = math.log(k[j]) + scipy.stats.chi2.logsf(xx, 2 * hp)
                assert abs(got[hp - 1, j] - sp) <= 1e-10 * max(1.0, abs(sp)), (hp, xx)
    assert np.isneginf(ora.log_significance(np.ones((1, 1)), np.array([0]), 1))[0, 0]


def test_dchi2_adjusted_restores_chi2_for_underestimated_errors():
    """Errors understated by 3x: the adjusted reduction is ~ Delta/9 (Section 3e)."""
    rng = np.random.default_rng(81)
    n, H = 400, 2
    t = np.sort(rng.uniform(0, 100, n))
    s = np.full(n, 0.1)
    x = 3 * s * rng.standard_normal(n)              # true noise 3x the stated sigma
    freqs = np.linspace(0.05, 3.0, 60)
    res = ora.dchi2(t, x, s, freqs, H)
    adj = ora.dchi2_adjusted(res["dchi2"], res["chi2_0"], n)
    ratio = res["dchi2"] / adj                      # = chi2_best / N_dof per row
    assert np.allclose(ratio, ratio[:, :1])
    assert 6.0 < ratio[1, 0] < 12.0                 # ~ 9 = (3x)^2
    best = np.argmax(res["dchi2"][1])
    np.testing.assert_allclose(adj[1, best], res["dchi2"][1, best] * (n - 5)
                               / (res["chi2_0"] - res["dchi2"][1, best]))


def test_top_candidates_hand_row():
    """Local maxima, plateau rule, eligibility and ln p ranking on a small row."""
    import math
    d = np.array([50.0, 1.0, 9.0, 2.0, 30.0, 30.0, 5.0, 7.0, 6.0, 40.0, 1.0, 3.0])
    freqs = np.arange(d.size) * 0.1
    idx, lp, dmax = ora.top_candidates(d, freqs, span=100.0, hp=1, K=10)
    # maxima: 2 (9), 4 (30; plateau counted at its left end), 7 (7), 9 (40); 11 is the last bin
    ref = sorted([(math.log(k) - d[k] / 2, k) for k in (2, 4, 7, 9)])
    assert list(idx) == [k for _, k in ref]
    np.testing.assert_allclose(lp, [v for v, _ in ref], rtol=1e-12)
    assert dmax == 40.0                          # bin 0 (50) is not eligible
    idx2, _, dmax2 = ora.top_candidates(d, freqs, span=100.0, hp=1, K=2, k_lo=5)
    assert list(idx2) == [9, 7] and dmax2 == 40.0
    idx3, _, _ = ora.top_candidates(d, freqs, span=3.0, hp=1, K=5)   # f >= 1/3 only
    assert list(idx3) == [9, 4, 7]


def test_floor_gridded_times():
    """Cell containment, identity on the grid, convergence to the exact search."""
    rng = np.random.default_rng(71)
    t, x, s = _rand_curve(rng, 80, span=40.0)
    df, L = 0.01, 4 * 512
    tq = ora.floor_gridded_times(t, df, L)
    dt = 1.0 / (df * L)
    assert np.all(tq <= t + 1e-12) and np.all(t - tq < dt * (1 + 1e-9))
    assert tq.min() == t.min()
    on_grid = t.min() + np.round((t - t.min()) / dt) * dt
    np.testing.assert_allclose(ora.floor_gridded_times(on_grid, df, L), on_grid, rtol=0,
                               atol=1e-9 * dt)
    freqs = np.array([0.21, 0.77, 1.9])
    exact = ora.dchi2(t, x, s, freqs, 2)["dchi2"]
    coarse = ora.dchi2(ora.floor_gridded_times(t, df, 256), x, s, freqs, 2)["dchi2"]
    fine = ora.dchi2(ora.floor_gridded_times(t, df, 1 << 20), x, s, freqs, 2)["dchi2"]
    assert np.max(np.abs(fine - exact)) < 1e-3 * np.max(np.abs(coarse - exact))


def test_detrend():
    """Removes polynomials exactly; residual weighted-orthogonal to t^j; degree 0
    is centring on the weighted mean."""
    rng = np.random.default_rng(81)
    t, x, s = _rand_curve(rng, 120, span=300.0, offset=2.45e6)
    w = 1.0 / s ** 2
    tau = (t - t.min()) / 100.0
    poly = 0.3 - 0.2 * tau + 0.05 * tau ** 2 - 0.004 * tau ** 3
    np.testing.assert_allclose(ora.detrend(t, poly, s, 3), 0.0, atol=1e-10)
    r = ora.detrend(t, x + poly, s, 3)
    for j in range(4):
        assert abs(np.sum(w * r * tau ** j)) <= 1e-8 * np.sum(w * np.abs(x) * tau ** j)
    r0 = ora.detrend(t, x, s, 0)
    np.testing.assert_allclose(r0, x - np.sum(w * x) / np.sum(w), atol=1e-12)
    # a trend leaves the periodogram's low frequencies once removed
    d_raw = ora.dchi2(t, x + 5 * poly, s, [0.004], 1)["dchi2"][0, 0]
    d_det = ora.dchi2(t, ora.detrend(t, x + 5 * poly, s, 3), s, [0.004], 1)["dchi2"][0, 0]
    assert d_det < 0.1 * d_raw


def test_scaled_condition_pins():
    """kappa of the diagonally scaled alpha (reading of the gate, Section 3a's
    low-frequency caveat): closed forms for 2x2, invariance under diagonal
    scaling, and the singular limit."""
    assert ora.scaled_condition(np.eye(5)) == pytest.approx(1.0, abs=1e-12)
    # A diagonal matrix is perfectly conditioned once scaled, however its
    # unscaled condition number (1e8 here) reads.
    assert ora.scaled_condition(np.diag([1.0, 1e8, 3.0])) == pytest.approx(1.0, abs=1e-12)
    for rho in (0.0, 0.3, -0.6, 0.99):
        a = np.array([[1.0, rho], [rho, 1.0]])
        want = (1.0 + abs(rho)) / (1.0 - abs(rho))
        assert ora.scaled_condition(a) == pytest.approx(want, rel=1e-12)
        # Scaling rows and columns by D leaves the scaled matrix unchanged.
        D = np.diag([3.0, 0.01])
        assert ora.scaled_condition(D @ a @ D) == pytest.approx(want, rel=1e-10)
    rng = np.random.default_rng(11)
    B = rng.standard_normal((40, 5))
    a = B.T @ B
    d = np.diag(rng.uniform(0.1, 100.0, 5))
    assert ora.scaled_condition(d @ a @ d) == pytest.approx(ora.scaled_condition(a), rel=1e-9)
    # Duplicated column: singular; a zero diagonal entry: infinite.
    M = np.stack([np.ones(6), np.arange(6.0), np.ones(6)], axis=1)
    assert ora.scaled_condition(M.T @ M) > 1e15
    assert ora.scaled_condition(np.diag([1.0, 0.0])) == np.inf


def test_gate_mask_hand_case():
    """Gate of the parity tolerance: k >= 1, f >= 1/span (inclusive), and
    kappa <= kappa_max (inclusive)."""
    freqs = np.array([0.0, 0.05, 0.0999, 0.1, 0.2, 0.3, 0.4])
    res = {"span": 10.0,
           "kappa": np.array([np.inf, 1.0, 1.0, 1.0, 100.0, 100.0 + 1e-9, np.nan])}
    got = ora.gate_mask(res, freqs, 100.0)
    np.testing.assert_array_equal(got, [False, False, False, True, True, False, False])
    # A curve with no span has no low-frequency cut, only the k = 0 and kappa ones.
    res0 = {"span": 0.0, "kappa": np.array([1.0, 1.0, 1e7])}
    np.testing.assert_array_equal(ora.gate_mask(res0, np.array([0.0, 1e-6, 5.0]), 1e6),
                                  [False, True, False])


def test_gate_agrees_with_flags_and_kappa():
    """On a real curve the gate drops exactly the DC and low-frequency bins the
    oracle flags, plus the bins whose scaled alpha is too ill-conditioned."""
    rng = np.random.default_rng(12)
    t, x, s = _rand_curve(rng, 60, span=20.0)
    freqs = np.linspace(0.0, 0.5, 41)
    res = ora.dchi2(t, x, s, freqs, 2)
    low = (res["flags"] & (ora.FLAG_DC | ora.FLAG_LOW_F)) != 0
    for kmax in (1e2, 1e6):
        g = ora.gate_mask(res, freqs, kmax)
        np.testing.assert_array_equal(g, ~low & (res["kappa"] <= kmax))
    # The low-frequency bins of this curve are the ones below 1/span.
    np.testing.assert_array_equal(low[1:], freqs[1:] < 1.0 / res["span"])
