"""Bare Green's function tables G0(tau) for impurity, finite and DCA clusters.

All functions return the "plus" propagator G0(tau) = <T c(tau) c^dagger(0)>_0
on 0 <= tau <= beta (entry 0 = the 0+ limit, entry -1 = the beta- limit).  For a
one-body level xi the plus propagator is exp(-tau*xi) * (1 - f(xi)), with f the
Fermi function; it is evaluated in an overflow-free form.

The model is the one of the paper, Sec. II A, Eq. (Ham): H0 contains the level
term -mu_tilde * n with mu_tilde = mu - U/2, so half filling of a bipartite
cluster is mu_tilde = 0.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np


def tau_grid(beta: float, n_tau: int) -> np.ndarray:
    """Uniform grid tau_m = m * beta / (n_tau - 1), m = 0 .. n_tau-1."""
    if n_tau < 2:
        raise ValueError("n_tau must be >= 2")
    return np.arange(n_tau, dtype=np.float64) * (beta / (n_tau - 1))


def fermi_weight(eps, tau, beta: float) -> np.ndarray:
    """exp(-tau*eps) / (1 + exp(-beta*eps)) for 0 <= tau <= beta, broadcast.

    Equals <c(tau) c^dagger> for a single level eps; never overflows because
    the exponent is kept non-positive in both branches.
    """
    eps = np.asarray(eps, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    # exponent -tau*eps - log(1 + e^{-beta*eps}) <= 0 for 0 <= tau <= beta
    return np.exp(-tau * eps - np.logaddexp(0.0, -beta * eps))


def semicircle_g0(beta: float, n_tau: int, mu_tilde: float = 0.0,
                  half_bandwidth: float = 2.0, n_quad: int = 4096) -> np.ndarray:
    """G0(tau) of a level coupled to a semicircular bath (Bethe lattice DMFT start).

    rho(eps) = sqrt(D^2 - eps^2) * 2 / (pi D^2) on |eps| <= D.  The integral
    int rho(eps) w(eps - mu_tilde, tau) d eps is done with Gauss-Chebyshev
    quadrature of the second kind (nodes x_i = cos(i pi/(M+1)), weights
    pi/(M+1) sin^2(i pi/(M+1)) for int sqrt(1-x^2) g(x) dx on [-1, 1]).
    """
    i = np.arange(1, n_quad + 1, dtype=np.float64)
    theta = i * np.pi / (n_quad + 1)
    x = np.cos(theta)
    w = np.pi / (n_quad + 1) * np.sin(theta) ** 2
    eps = half_bandwidth * x
    weights = (2.0 / np.pi) * w  # int rho(eps) g(eps) deps = (2/pi) int sqrt(1-x^2) g(Dx) dx
    taus = tau_grid(beta, n_tau)
    out = np.zeros(n_tau, dtype=np.float64)
    chunk = 512
    for a in range(0, n_tau, chunk):
        t = taus[a:a + chunk]
        out[a:a + chunk] = fermi_weight(eps[None, :] - mu_tilde, t[:, None], beta) @ weights
    return out


def finite_system_g0(h1: np.ndarray, beta: float, n_tau: int,
                     orbitals: list[int] | None = None) -> np.ndarray:
    """Exact G0_xy(tau) of a finite one-body Hamiltonian h1 (real symmetric).

    Returns an array [len(orbitals), len(orbitals), n_tau]; `orbitals` are the
    interacting (cluster) orbitals, by default all of them.
    """
    h1 = np.asarray(h1, dtype=np.float64)
    eps, phi = np.linalg.eigh(h1)
    if orbitals is None:
        orbitals = list(range(h1.shape[0]))
    ph = phi[orbitals, :]  # [nc, n_levels]
    taus = tau_grid(beta, n_tau)
    w = fermi_weight(eps[:, None], taus[None, :], beta)  # [levels, tau]
    return np.einsum("xa,ya,at->xyt", ph, ph, w)


@dataclass
class Cluster:
    """A periodic cluster: sites of the superlattice cell and cluster momenta."""
    superlattice: np.ndarray   # [d, d] integer rows a_i
    sites: np.ndarray          # [Nc, d] integer lattice points in the cell
    momenta: np.ndarray        # [Nc, d] cluster momenta K in [0, 2 pi)
    site_disp: np.ndarray      # [Nc, Nc] int32: index of the site r_x - r_y (reduced)

    @property
    def n_sites(self) -> int:
        return self.sites.shape[0]


def _reduce(points: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Reduce integer lattice points into the superlattice cell spanned by rows of a."""
    ainv = np.linalg.inv(a.astype(np.float64))
    f = points.astype(np.float64) @ ainv
    f = f - np.floor(f + 1e-9)
    return np.rint(f @ a).astype(np.int64)


_CLUSTER_CACHE: dict = {}


def make_cluster(superlattice) -> Cluster:
    key = tuple(map(tuple, np.asarray(superlattice, dtype=np.int64).tolist()))
    if key not in _CLUSTER_CACHE:
        _CLUSTER_CACHE[key] = _make_cluster(superlattice)
    return _CLUSTER_CACHE[key]


def _make_cluster(superlattice) -> Cluster:
    a = np.asarray(superlattice, dtype=np.int64)
    d = a.shape[0]
    nc = int(round(abs(np.linalg.det(a.astype(np.float64)))))
    corners = np.array([np.array(c) @ a for c in itertools.product([0, 1], repeat=d)])
    lo, hi = corners.min(axis=0), corners.max(axis=0)
    box = np.array(list(itertools.product(*[range(lo[i], hi[i] + 1) for i in range(d)])))
    red = _reduce(box, a)
    uniq = sorted({tuple(r) for r in red})
    sites = np.array(uniq, dtype=np.int64)
    if sites.shape[0] != nc:
        raise ValueError(f"cluster enumeration found {sites.shape[0]} sites, expected {nc}")
    # canonical order: origin first, then lexicographic
    index = {tuple(r): i for i, r in enumerate(sites)}
    disp = np.zeros((nc, nc), dtype=np.int32)
    for x in range(nc):
        dif = _reduce(sites[x][None, :] - sites, a)
        for y in range(nc):
            disp[x, y] = index[tuple(dif[y])]
    # cluster momenta: K = 2 pi a^{-1} m (m integer), reduced mod 2 pi.  They form
    # a group of order nc generated by the unit vectors m = e_i: breadth-first
    # closure under adding e_i.
    ainv = np.linalg.inv(a.astype(np.float64))

    def _k_of(m):
        k = 2 * np.pi * (ainv @ np.array(m, dtype=np.float64))
        k = np.mod(k, 2 * np.pi)
        k[np.isclose(k, 2 * np.pi, atol=1e-9)] = 0.0
        return tuple(np.round(k, 9))

    ks = {_k_of([0] * d)}
    frontier = [[0] * d]
    while frontier and len(ks) <= nc:
        nxt = []
        for m in frontier:
            for i in range(d):
                m2 = list(m)
                m2[i] += 1
                key = _k_of(m2)
                if key not in ks:
                    ks.add(key)
                    nxt.append(m2)
        frontier = nxt
    momenta = np.array(sorted(ks), dtype=np.float64)
    if momenta.shape[0] != nc:
        raise ValueError("cluster momentum enumeration failed")
    return Cluster(superlattice=a, sites=sites, momenta=momenta, site_disp=disp)


def _dispersion(k: np.ndarray, t: float) -> np.ndarray:
    return -2.0 * t * np.cos(k).sum(axis=-1)


_PATCH_CACHE: dict = {}


def _patch_weights(cluster: Cluster, n_fine: int):
    """Fine-mesh k points and their (tie-split) assignment to cluster momenta."""
    key = (cluster.superlattice.tobytes(), cluster.superlattice.shape, n_fine)
    if key not in _PATCH_CACHE:
        _PATCH_CACHE[key] = _patch_weights_uncached(cluster, n_fine)
    return _PATCH_CACHE[key]


def _patch_weights_uncached(cluster: Cluster, n_fine: int):
    d = cluster.sites.shape[1]
    grid = np.array(list(itertools.product(range(n_fine), repeat=d)), dtype=np.float64)
    kf = 2 * np.pi * grid / n_fine
    imgs = np.array(list(itertools.product([-1, 0, 1], repeat=d)), dtype=np.float64) * 2 * np.pi
    kimg = (cluster.momenta[:, None, :] + imgs[None, :, :])  # [Nc, nimg, d]
    dist = np.linalg.norm(kf[:, None, None, :] - kimg[None, :, :, :], axis=-1).min(axis=2)
    dmin = dist.min(axis=1, keepdims=True)
    w = (dist <= dmin + 1e-9).astype(np.float64)
    w /= w.sum(axis=1, keepdims=True)
    return kf, w  # w: [n_fine^d, Nc], rows sum to 1


def cluster_density(mu_tilde: float, cluster: Cluster, beta: float, t: float = 1.0,
                    n_fine: int = 64) -> float:
    """Non-interacting density per site (both spins) of the lattice, -mu_tilde level."""
    d = cluster.sites.shape[1]
    grid = np.array(list(itertools.product(range(n_fine), repeat=d)), dtype=np.float64)
    xi = _dispersion(2 * np.pi * grid / n_fine, t) - mu_tilde
    return float(2.0 * fermi_weight(-xi, 0.0, beta).mean())  # f(xi) = w(-xi, 0)


def solve_mu_for_density(density: float, cluster: Cluster, beta: float, t: float = 1.0,
                         n_fine: int = 64) -> float:
    lo, hi = -20.0 * t, 20.0 * t
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if cluster_density(mid, cluster, beta, t, n_fine) < density:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def dca_cluster_g0(cluster: Cluster, beta: float, n_tau: int, mu_tilde: float,
                   t: float = 1.0, n_fine: int = 64) -> np.ndarray:
    """DCA coarse-grained bare G0 (zero self-energy) per displacement class.

    G0(K, tau) is the patch average of the lattice plus-propagator of the
    nearest-neighbour tight-binding band; G0(X, tau) = (1/Nc) sum_K cos(K.X)
    G0(K, tau).  Returns [Nc, n_tau], row j = displacement of cluster site j.
    """
    kf, w = _patch_weights(cluster, n_fine)
    xi = _dispersion(kf, t) - mu_tilde
    wn = w / w.sum(axis=0, keepdims=True)           # patch averages
    taus = tau_grid(beta, n_tau)
    gk = np.zeros((cluster.n_sites, n_tau), dtype=np.float64)
    chunk = 256
    for a in range(0, n_tau, chunk):
        f = fermi_weight(xi[:, None], taus[None, a:a + chunk], beta)  # [nk, chunk]
        gk[:, a:a + chunk] = wn.T @ f
    phase = np.cos(cluster.sites.astype(np.float64) @ cluster.momenta.T)  # [X, K]
    return (phase @ gk) / cluster.n_sites
