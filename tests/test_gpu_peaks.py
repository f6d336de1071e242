"""fchi2_top_peaks (the K largest strict local maxima of one Delta chi2 row,
ties to the lower bin) on rows written directly, against the same rule
applied on the host: the largest grid (2^24 bins, 1024 blocks, so every
thread of the merge holds four block lists), several curves and rows, values
quantised so that equal values are common, and rows with fewer than K maxima
(the rest -1)."""
import numpy as np
import pytest

from paper_0901_1913_amd import fchi2 as F
from tests.gpu_util import note

pytestmark = pytest.mark.gpu


def _host(row, k_lo, K):
    k = np.arange(k_lo, row.shape[0] - 1)
    is_max = (row[k] > row[k - 1]) & (row[k] >= row[k + 1])
    cand = k[is_max]
    order = np.lexsort((cand, -row[cand].astype(np.float64)))
    out = np.full(K, -1, dtype=np.int64)
    sel = cand[order][:K]
    out[:len(sel)] = sel
    return out


def _plan(n_curves, H, n_freq):
    off = np.arange(n_curves + 1, dtype=np.int64) * 50
    return F.Plan(off, 10.0, H, n_freq, precision="mixed")


@pytest.mark.parametrize("n_freq,K,levels", [(2 ** 24, 64, 1000), (2 ** 22, 16, 50),
                                             (2 ** 14, 64, 7)])
def test_top_peaks_match_the_host_rule(n_freq, K, levels):
    import torch
    nc, H, hrow, k_lo = 3, 2, 1, 5
    note(f"top peaks: n_freq 2^{int(np.log2(n_freq))}, K {K}, {levels} value levels")
    plan = _plan(nc, H, n_freq)
    g = torch.Generator(device="cuda").manual_seed(int(np.log2(n_freq)) * 100 + K)
    d = torch.floor(torch.rand((nc, H, n_freq), generator=g, device="cuda") * levels)
    idx = plan.top_peaks(d, hrow, k_lo, K)
    torch.cuda.synchronize()
    got = idx.cpu().numpy()
    dn = d.cpu().numpy()
    for c in range(nc):
        want = _host(dn[c, hrow], k_lo, K)
        assert np.array_equal(got[c], want), (c, got[c][:8], want[:8])
    plan.close()


def test_top_peaks_fewer_maxima_than_k():
    import torch
    n_freq, K = 2 ** 16, 64
    note("top peaks: rows with 0, 1 and 4 strict local maxima")
    plan = _plan(3, 1, n_freq)
    d = torch.arange(n_freq, dtype=torch.float32, device="cuda").repeat(3, 1, 1)  # increasing
    d[1, 0, 1000] = 1e9                       # one maximum
    for j, k in enumerate((77, 5000, 5001, 40000, 65000)):
        d[2, 0, k] = 1e6 + j                  # four (5000 is not one: 5001 is larger)
    d[2, 0, 5002] = 0.0
    idx = plan.top_peaks(d, 0, 1, K).cpu().numpy()
    dn = d.cpu().numpy()
    for c in range(3):
        assert np.array_equal(idx[c], _host(dn[c, 0], 1, K)), (c, idx[c][:6])
    assert (idx[0] == -1).all()
    assert idx[1][0] == 1000 and (idx[1][1:] == -1).all()
    assert list(idx[2][:4]) == [65000, 40000, 5001, 77] and (idx[2][4:] == -1).all()
    plan.close()
