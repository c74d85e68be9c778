"""Named synthetic workloads: model parameters plus G0 tables.

Every workload is deterministic given its arguments (the batched mix draws
its per-chain parameters from a seeded numpy Generator).  A Workload carries
what both implementations take as input: beta, U, K, the cluster size, the
site-pair -> table map and one G0 table set per spin sector.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .g0 import (dca_cluster_g0, finite_system_g0, make_cluster, semicircle_g0,
                 solve_mu_for_density)


@dataclass
class Workload:
    name: str
    beta: float
    U: float
    K: float
    n_sites: int
    site_disp: np.ndarray          # int32 [n_sites * n_sites]
    g0_up: np.ndarray              # float64 [n_disp, n_tau]
    g0_dn: np.ndarray              # float64 [n_disp, n_tau]
    meta: dict = field(default_factory=dict)
    site_pos: np.ndarray | None = None   # [n_sites, 3] positions r_x (momentum measurement)
    kvecs: np.ndarray | None = None      # [n_k, 3] cluster momenta K

    @property
    def n_tau(self) -> int:
        return int(self.g0_up.shape[1])

    @property
    def n_disp(self) -> int:
        return int(self.g0_up.shape[0])

    def __post_init__(self):
        self.site_disp = np.ascontiguousarray(self.site_disp, dtype=np.int32).reshape(-1)
        self.g0_up = np.ascontiguousarray(self.g0_up, dtype=np.float64)
        self.g0_dn = np.ascontiguousarray(self.g0_dn, dtype=np.float64)
        if self.g0_up.ndim == 1:
            self.g0_up = self.g0_up[None, :]
            self.g0_dn = self.g0_dn[None, :]
        assert self.site_disp.size == self.n_sites * self.n_sites
        assert self.g0_up.shape == self.g0_dn.shape
        assert int(self.site_disp.max()) < self.n_disp
        if self.site_pos is not None:
            self.site_pos = _pad3(self.site_pos)
            self.kvecs = _pad3(self.kvecs)
            assert self.site_pos.shape[0] == self.n_sites


def _pad3(a) -> np.ndarray:
    """Rows of 1-3 coordinates as rows of 3 (missing dimensions zero)."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    out = np.zeros((a.shape[0], 3))
    out[:, :a.shape[1]] = a
    return np.ascontiguousarray(out)


def anderson_semicircle(beta=10.0, U=4.0, K=1.0, n_tau=4096, mu_tilde=0.0) -> Workload:
    """Single-site Anderson impurity, semicircular bath of half-bandwidth 2."""
    g = semicircle_g0(beta, n_tau, mu_tilde=mu_tilde)
    return Workload("anderson_semicircle", beta, U, K, 1, np.zeros(1, np.int32), g, g.copy(),
                    {"mu_tilde": mu_tilde, "half_bandwidth": 2.0})


def hubbard_atom(beta=10.0, U=4.0, K=1.0, n_tau=1024) -> Workload:
    """Isolated Hubbard atom at half filling: G0(tau) = 1/2 for all tau."""
    g = np.full(n_tau, 0.5)
    return Workload("hubbard_atom", beta, U, K, 1, np.zeros(1, np.int32), g, g.copy())


def _finite_tables(g0xy: np.ndarray):
    nc = g0xy.shape[0]
    tables = g0xy.reshape(nc * nc, -1)
    disp = np.arange(nc * nc, dtype=np.int32)
    return tables, disp


def hubbard_dimer(beta=2.0, U=2.0, K=1.0, t=1.0, mu_tilde=0.0, n_tau=2048) -> Workload:
    """Isolated two-site Hubbard cluster (each site pair has its own table)."""
    h1 = np.array([[-mu_tilde, -t], [-t, -mu_tilde]])
    g = finite_system_g0(h1, beta, n_tau)
    tables, disp = _finite_tables(g)
    return Workload("hubbard_dimer", beta, U, K, 2, disp, tables, tables.copy(),
                    {"h1": h1, "t": t, "mu_tilde": mu_tilde},
                    site_pos=[[0.0], [1.0]], kvecs=[[0.0], [np.pi]])


def hubbard_plaquette(beta=8.0, U=6.0, K=1.0, t=1.0, tp=0.4, mu_tilde=-1.2, n_tau=2048) -> Workload:
    """Isolated 2x2 Hubbard plaquette with nearest (t) and diagonal (tp)
    hopping; every site pair has its own table.  Away from half filling with
    tp != 0 the auxiliary-field weights take both signs."""
    h1 = np.zeros((4, 4))
    for a, b in ((0, 1), (1, 3), (3, 2), (2, 0)):
        h1[a, b] = h1[b, a] = -t
    for a, b in ((0, 3), (1, 2)):
        h1[a, b] = h1[b, a] = -tp
    h1 -= mu_tilde * np.eye(4)
    g = finite_system_g0(h1, beta, n_tau)
    tables, disp = _finite_tables(g)
    return Workload("hubbard_plaquette", beta, U, K, 4, disp, tables, tables.copy(),
                    {"h1": h1, "t": t, "tp": tp, "mu_tilde": mu_tilde},
                    site_pos=[[0, 0], [1, 0], [0, 1], [1, 1]],
                    kvecs=[[0, 0], [np.pi, 0], [0, np.pi], [np.pi, np.pi]])


def anderson_bath(beta=4.0, U=3.0, K=1.0, v=0.7, eps_bath=(-1.0, 1.0), mu_tilde=0.0,
                  n_tau=2048) -> Workload:
    """Impurity (orbital 0) hybridised with a few bath levels; Nc = 1."""
    nb = len(eps_bath)
    h1 = np.zeros((nb + 1, nb + 1))
    h1[0, 0] = -mu_tilde
    for p, e in enumerate(eps_bath):
        h1[p + 1, p + 1] = e
        h1[0, p + 1] = h1[p + 1, 0] = v
    g = finite_system_g0(h1, beta, n_tau, orbitals=[0])[0, 0]
    return Workload("anderson_bath", beta, U, K, 1, np.zeros(1, np.int32), g, g.copy(),
                    {"h1": h1, "v": v, "eps_bath": list(eps_bath), "mu_tilde": mu_tilde})


def dca_square(L=4, beta=8.0, U=8.0, K=1.0, density=None, n_tau=8192, t=1.0,
               n_fine=64, superlattice=None) -> Workload:
    """2D Hubbard DCA cluster; zero-self-energy coarse-grained G0.

    density None means half filling (mu_tilde = 0); otherwise mu_tilde is
    fixed by bisection on the non-interacting lattice density.
    """
    sl = superlattice if superlattice is not None else [[L, 0], [0, L]]
    cl = make_cluster(sl)
    mu = 0.0 if density is None else solve_mu_for_density(density, cl, beta, t, n_fine)
    g = dca_cluster_g0(cl, beta, n_tau, mu, t, n_fine)
    return Workload(f"dca_square_{cl.n_sites}", beta, U, K, cl.n_sites, cl.site_disp, g,
                    g.copy(), {"mu_tilde": mu, "superlattice": np.asarray(sl).tolist(),
                               "density": density, "t": t, "n_fine": n_fine},
                    site_pos=cl.sites, kvecs=cl.momenta)


def dca_cubic(beta=6.0, U=8.0, K=1.0, n_tau=8192, t=1.0, n_fine=20,
              superlattice=((5, 5, 0), (5, -5, 0), (0, 0, 2))) -> Workload:
    """3D Hubbard DCA cluster at half filling (default Nc = 100, bipartite)."""
    cl = make_cluster(superlattice)
    g = dca_cluster_g0(cl, beta, n_tau, 0.0, t, n_fine)
    return Workload(f"dca_cubic_{cl.n_sites}", beta, U, K, cl.n_sites, cl.site_disp, g,
                    g.copy(), {"mu_tilde": 0.0, "superlattice": np.asarray(superlattice).tolist(),
                               "t": t, "n_fine": n_fine},
                    site_pos=cl.sites, kvecs=cl.momenta)


_MIX_LATTICES = {
    4: [[2, 0], [0, 2]],
    8: [[2, 2], [2, -2]],
    16: [[4, 0], [0, 4]],
    32: [[4, 4], [4, -4]],
}


def batched_mix(n_chains=512, seed=0, n_tau=4096, n_fine=32, K=1.0):
    """Per-chain workloads for the batched form: Nc in {4,8,16,32}, beta in
    [4, 12], U in [4, 8], half filling.  Tables are shared between chains with
    identical (Nc, beta) only through Python object identity, never copied.
    """
    rng = np.random.default_rng(seed)
    ncs = rng.choice(sorted(_MIX_LATTICES), size=n_chains)
    betas = rng.uniform(4.0, 12.0, size=n_chains)
    us = rng.uniform(4.0, 8.0, size=n_chains)
    out = []
    for c in range(n_chains):
        nc = int(ncs[c])
        w = dca_square(beta=float(betas[c]), U=float(us[c]), K=K, n_tau=n_tau,
                       n_fine=n_fine, superlattice=_MIX_LATTICES[nc])
        w.name = f"mix{c}_nc{nc}"
        out.append(w)
    return out


def named_workload(name: str, **kw) -> Workload:
    table = {
        "anderson_semicircle": anderson_semicircle,
        "hubbard_atom": hubbard_atom,
        "hubbard_dimer": hubbard_dimer,
        "hubbard_plaquette": hubbard_plaquette,
        "anderson_bath": anderson_bath,
        "dca_square": dca_square,
        "dca_cubic": dca_cubic,
    }
    return table[name](**kw)
