"""The identity behind the GPU's folded inverse transforms (CPU): a shell of
lags is closed under a change of sign of any component, so the shell sums of
S2 need R_h only summed over the lags that fold to f = (|hx|, |hy|, |hz|),

    X(f) = sum_{h -> f} R_h = N^-6 sum_k Psi(k) prod_a mu(f_a) cos(2 pi k_a f_a / N),

with mu = 1 at f_a = 0 and N/2 and 2 between (the number of lags behind f_a).
Written here with plain numpy cosine matrices and compared with the oracle's
structure function (eq. (SF_single_spec2)) on random fields, and the lag
multiplicities with the shell sizes."""
import numpy as np
import pytest

import oracle


def folded_structure_function(u):
    n = u.shape[1]
    half = n // 2
    psi = sum(np.abs(np.fft.fftn(u[a])) ** 2 for a in range(3))
    f = np.arange(half + 1)
    mu = np.where((f == 0) | (f == half), 1.0, 2.0)
    c = mu[:, None] * np.cos(2 * np.pi * np.outer(f, np.arange(n)) / n)      # [f, k]
    x = np.einsum("az,by,cx,zyx->abc", c, c, c, psi) / n ** 6                # X(f)
    r0 = psi.sum() / n ** 6
    lags = mu[:, None, None] * mu[None, :, None] * mu[None, None, :]
    shell = np.floor(np.sqrt(f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2) + 0.5)
    s2 = np.empty(half)
    for r in range(1, half + 1):
        sel = shell == r
        s2[r - 1] = np.sum(2.0 * (lags[sel] * r0 - x[sel])) / np.sum(lags[sel])
    return s2, lags, shell


@pytest.mark.parametrize("n,seed", [(8, 1), (16, 2), (32, 3)])
def test_folded_sums_give_the_oracle_structure_function(n, seed):
    u = np.random.default_rng(seed).standard_normal((3, n, n, n))
    s2, _, _ = folded_structure_function(u)
    s2o = oracle.structure_function(u)
    assert np.max(np.abs(s2 - s2o)) <= 1e-12 * np.max(np.abs(s2o))


@pytest.mark.parametrize("n", [8, 16])
def test_folded_lags_count_every_lag_once(n):
    """The multiplicities mu(f) add up to the N^3 lags, and per shell to the
    number of minimum-image lags whose length rounds to it."""
    _, lags, shell = folded_structure_function(np.zeros((3, n, n, n)))
    assert lags.sum() == n ** 3
    h = np.fft.fftfreq(n) * n
    h[h == -n // 2] = n // 2
    hz, hy, hx = np.meshgrid(h, h, h, indexing="ij")
    full = np.floor(np.sqrt(hx ** 2 + hy ** 2 + hz ** 2) + 0.5)
    for r in range(0, int(full.max()) + 1):
        assert lags[shell == r].sum() == np.count_nonzero(full == r), r
