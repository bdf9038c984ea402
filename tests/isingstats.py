"""Binning + jackknife estimates of e and C_V from an energy time series (test helper)."""
import numpy as np


def estimates(E, N, beta, n_bins=20):
    """e = -<E>/N and C_V = beta^2 (<E^2> - <E>^2)/N with jackknife errors over n_bins bins."""
    E = np.asarray(E, dtype=np.float64)
    m = len(E) // n_bins
    E = E[:m * n_bins].reshape(n_bins, m)
    s1 = E.sum(axis=1)
    s2 = (E * E).sum(axis=1)
    tot1, tot2, n = s1.sum(), s2.sum(), m * n_bins

    def obs(a1, a2, cnt):
        mean = a1 / cnt
        return -mean / N, beta * beta * (a2 / cnt - mean * mean) / N

    e, c = obs(tot1, tot2, n)
    jk = np.array([obs(tot1 - s1[b], tot2 - s2[b], n - m) for b in range(n_bins)])
    var = (n_bins - 1) / n_bins * ((jk - jk.mean(axis=0)) ** 2).sum(axis=0)
    return e, float(np.sqrt(var[0])), c, float(np.sqrt(var[1]))
