"""Seeded synthetic inputs (shared by tests, bench and smoke; no operator arithmetic).

Perturbed Maxwellian cells: c_alpha = delta_{alpha,000} + sigma_kl xi_alpha with
xi ~ N(0, 1) i.i.d. for every mode (the unit Maxwellian included) and
sigma_kl = sigma0 exp(-(k + l)/2), sigma0 = 0.05.  Draws use NumPy's PCG64 with
the stated seed; row b of the (B, N) matrix is cell b.
"""
import numpy as np

BASE_SEED = 20260528


def mode_kl(K, L):
    """Per flat mode n = q*(K+1) + k: arrays (k, l, m)."""
    NK = K + 1
    ks, ls, ms = [], [], []
    for l in range(L + 1):
        for m in range(-l, l + 1):
            for k in range(NK):
                ks.append(k); ls.append(l); ms.append(m)
    return np.array(ks), np.array(ls), np.array(ms)


def perturbed_maxwellian(K, L, B, seed, sigma0=0.05):
    """The seeded (B, N) coefficient matrix, float64."""
    k, l, _ = mode_kl(K, L)
    sigma = sigma0 * np.exp(-0.5 * (k + l))
    N = len(k)
    rng = np.random.Generator(np.random.PCG64(seed))
    xi = rng.standard_normal((B, N))
    c = sigma[None, :] * xi
    c[:, 0] += 1.0
    return c


def unit_maxwellian(K, L, B=1):
    c = np.zeros((B, (K + 1) * (L + 1) ** 2))
    c[:, 0] = 1.0
    return c


# The five workloads (sizes and models) that the tests and the benchmark use.
WORKLOADS = {
    "single_cell": dict(name="hs_fp64_K3L3_single", model="hs", gamma=1.0, K=3, L=3, B=1, seed=BASE_SEED + 1),
    "k8_batch": dict(name="mm_hs_K8L8_B4096", model=("mm", "hs"), K=8, L=8, B=4096, seed=BASE_SEED + 2),
    "k12_batch": dict(name="vhs0.5_K12L12_B65536", model="vhs", gamma=0.5, K=12, L=12, B=65536, seed=BASE_SEED + 3),
    "uneven": dict(name="uneven_20000_K4-16_hs_vhs", cells=20000, sizes=(4, 8, 12, 16), seed=BASE_SEED + 4),
    "serving": dict(name="serving_poisson_2000rps", rate=2000.0, sizes=(8, 12, 16), max_cells=4096, seed=BASE_SEED + 5),
}
