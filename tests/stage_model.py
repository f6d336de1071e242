"""FP64 numpy model of the fast method's stages (test helper only).

It mirrors the stage structure of the HIP path (kernel spreading on grids of
L = 4 n_freq cells per harmonic multiple, FFT with the +i sign, division by the
kernel's Fourier transform, product-to-sum assembly, prefix Cholesky) so that
conventions can be checked on the CPU against the oracle.  It is neither the
oracle nor part of the product.
"""
import numpy as np


def es_phi(z, beta):
    out = np.zeros_like(z)
    m = np.abs(z) < 1.0
    out[m] = np.exp(beta * (np.sqrt(1.0 - z[m] ** 2) - 1.0))
    return out


def spread(pos, s, L, w, beta):
    g = np.zeros(L)
    hw = w // 2
    fl = np.floor(pos)
    for dj in range(-hw - 1, hw + 2):
        j = fl + dj
        phi = es_phi((j - pos) * (2.0 / w), beta)
        np.add.at(g, j.astype(np.int64) % L, s * phi)
    return g


def phi_hat(k, L, w, beta, n_gl=128):
    x, wt = np.polynomial.legendre.leggauss(n_gl)
    pos = x > 0
    x, wt = x[pos], wt[pos]
    a = np.pi * w * np.asarray(k, dtype=np.float64)[:, None] / L
    return (w * wt * np.exp(beta * (np.sqrt(1 - x * x) - 1)) * np.cos(a * x)).sum(axis=1)


def transforms(t, x, sigma, f_max, H, n_freq, w=14):
    """Q_m[k] (m = 0..2H) and P_m[k] (m = 0..H) from the gridded data."""
    L = 4 * n_freq
    df = f_max / n_freq
    beta = 2.30 * w
    c_off = w // 2 + 2
    wt = 1.0 / sigma ** 2
    W = wt.sum()
    xbar = (wt * x).sum() / W
    y = x - xbar
    v = (t - t[0]) * df
    k = np.arange(n_freq)
    D = np.exp(-2j * np.pi * ((k * c_off) % L) / L) / phi_hat(k, L, w, beta)
    Q = np.zeros((2 * H + 1, n_freq), dtype=complex)
    P = np.zeros((H + 1, n_freq), dtype=complex)
    Q[0] = W
    for m in range(1, 2 * H + 1):
        pos = (m * v) * L + c_off
        Q[m] = (np.fft.ifft(spread(pos, wt, L, w, beta)) * L)[:n_freq] * D
        if m <= H:
            P[m] = (np.fft.ifft(spread(pos, wt * y, L, w, beta)) * L)[:n_freq] * D
    return Q, P, W


def assemble(Qk, Pk, H):
    """alpha, beta at one bin from Q_m, P_m via the product-to-sum identities."""
    d = 2 * H + 1

    def Cp(g):
        return Qk[abs(g)].real

    def Sp(g):
        return np.sign(g) * Qk[abs(g)].imag if g != 0 else 0.0

    a = np.zeros((d, d))
    b = np.zeros(d)
    a[0, 0] = Qk[0].real
    for h in range(1, H + 1):
        a[2 * h - 1, 0] = a[0, 2 * h - 1] = Qk[h].imag
        a[2 * h, 0] = a[0, 2 * h] = Qk[h].real
        b[2 * h - 1] = Pk[h].imag
        b[2 * h] = Pk[h].real
        for hp in range(1, H + 1):
            a[2 * h - 1, 2 * hp - 1] = 0.5 * (Cp(h - hp) - Cp(h + hp))
            a[2 * h - 1, 2 * hp] = 0.5 * (Sp(h + hp) + Sp(h - hp))
            a[2 * h, 2 * hp - 1] = 0.5 * (Sp(h + hp) - Sp(h - hp))
            a[2 * h, 2 * hp] = 0.5 * (Cp(h - hp) + Cp(h + hp))
    return a, b


def dchi2(t, x, sigma, f_max, H, n_freq, w=14, bins=None):
    Q, P, W = transforms(t, x, sigma, f_max, H, n_freq, w)
    bins = np.arange(1, n_freq) if bins is None else np.asarray(bins)
    out = np.zeros((H, bins.shape[0]))
    for j, k in enumerate(bins):
        a, b = assemble(Q[:, k], P[:, k], H)
        Lc = np.linalg.cholesky(a)
        z = np.linalg.solve(Lc, b)
        acc = np.cumsum(z * z)
        out[:, j] = acc[2::2]
    return out
