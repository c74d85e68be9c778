"""Fock-space brute force for tiny systems (test infrastructure).

Independent of both CT-AUX implementations: it builds fermion operators by
Jordan-Wigner on the full Fock space of L orbitals x 2 spins and evaluates
  * thermal averages of the interacting Hamiltonian H = H0 + V (paper Eq. (Ham),
    with V = U sum_x [n_x,up n_x,dn - (n_x,up + n_x,dn)/2] on interacting sites x),
  * the imaginary-time Green's function G_xy(tau) = <T c_x(tau) c_y^dagger(0)>,
  * the time-ordered trace Z_n({s_i, tau_i}) of Eq. (Zn) for a given
    auxiliary-spin configuration, and ratios with an extra c c^dagger pair.
Everything uses dense matrices and eigendecompositions; sizes are 4^L.
"""

from __future__ import annotations

import numpy as np


class Fock:
    def __init__(self, n_orb: int):
        self.n_orb = n_orb
        self.n_modes = 2 * n_orb          # mode = 2*orb + spin, spin 0 = up, 1 = down
        self.dim = 2 ** self.n_modes
        self.c = [self._annihilator(m) for m in range(self.n_modes)]
        self.n = [self.c[m].T @ self.c[m] for m in range(self.n_modes)]
        self.eye = np.eye(self.dim)

    def _annihilator(self, m: int) -> np.ndarray:
        dim = self.dim
        op = np.zeros((dim, dim))
        for state in range(dim):
            if state >> m & 1:
                sign = (-1) ** bin(state & ((1 << m) - 1)).count("1")
                op[state ^ (1 << m), state] = sign
        return op

    def mode(self, orb: int, spin: int) -> int:
        return 2 * orb + spin

    def h0(self, h1: np.ndarray) -> np.ndarray:
        H = np.zeros((self.dim, self.dim))
        for s in range(2):
            for a in range(self.n_orb):
                for b in range(self.n_orb):
                    if h1[a, b] != 0.0:
                        ca = self.c[self.mode(a, s)]
                        cb = self.c[self.mode(b, s)]
                        H += h1[a, b] * (ca.T @ cb)
        return H

    def interaction(self, U: float, sites) -> np.ndarray:
        V = np.zeros((self.dim, self.dim))
        for x in sites:
            nu, nd = self.n[self.mode(x, 0)], self.n[self.mode(x, 1)]
            V += U * (nu @ nd - 0.5 * (nu + nd))
        return V


def expm_sym(H: np.ndarray, t: float) -> np.ndarray:
    e, v = np.linalg.eigh(H)
    e0 = e.min()
    return (v * np.exp(-t * (e - e0))) @ v.T, e0


class ED:
    """Thermal properties of H0 + V for a small system."""

    def __init__(self, h1: np.ndarray, U: float, beta: float, sites):
        self.f = Fock(h1.shape[0])
        self.beta = beta
        self.sites = list(sites)
        self.H0 = self.f.h0(h1)
        self.V = self.f.interaction(U, self.sites)
        self.H = self.H0 + self.V
        self.e, self.v = np.linalg.eigh(self.H)
        self.w = np.exp(-beta * (self.e - self.e.min()))
        self.Z = self.w.sum()

    def avg(self, op: np.ndarray) -> float:
        d = np.einsum("ia,ij,ja->a", self.v, op, self.v)
        return float((self.w * d).sum() / self.Z)

    def double_occ(self, x: int) -> float:
        f = self.f
        return self.avg(f.n[f.mode(x, 0)] @ f.n[f.mode(x, 1)])

    def density(self, x: int, spin: int) -> float:
        return self.avg(self.f.n[self.f.mode(x, spin)])

    def potential(self) -> float:
        return self.avg(self.V)

    def greens(self, x: int, y: int, spin: int, tau: float) -> float:
        """<T c_x(tau) c_y^dagger(0)> for 0 < tau < beta."""
        f = self.f
        cx = self.v.T @ f.c[f.mode(x, spin)] @ self.v
        cy = self.v.T @ f.c[f.mode(y, spin)].T @ self.v
        e = self.e - self.e.min()
        left = np.exp(-(self.beta - tau) * e)
        right = np.exp(-tau * e)
        return float(np.einsum("a,ab,b,ba->", left, cx, right, cy) / self.Z)


    def greens_matsubara(self, x: int, y: int, spin: int, omega: float) -> complex:
        """int_0^beta e^{i omega tau} <T c_x(tau) c_y^dagger(0)> d tau for a fermionic
        omega (Lehmann):  -(1/Z) sum_mn (e^{-beta E_n} + e^{-beta E_m}) <m|c_x|n><n|c_y^+|m>
        / (i omega + E_m - E_n)."""
        f = self.f
        cx = self.v.T @ f.c[f.mode(x, spin)] @ self.v
        cy = self.v.T @ f.c[f.mode(y, spin)].T @ self.v
        e = self.e - self.e.min()
        w = np.exp(-self.beta * e)
        num = (w[None, :] + w[:, None]) * cx * cy.T          # [m, n]
        den = 1j * omega + e[:, None] - e[None, :]
        return complex(-(num / den).sum() / self.Z)


def vertex_product(f: Fock, H0: np.ndarray, beta: float, gamma: float, verts,
                   extra=None) -> float:
    """Tr of the time-ordered product of Eq. (Zn).

    verts: list of (tau, site, s).  extra: optional list of (tau, op) inserted
    at their times (for the G(tau, 0) pin); operators at equal time keep the
    order given (earlier in the list = further right).
    """
    items = [(t, "v", (x, s)) for (t, x, s) in verts]
    if extra:
        items += [(t, "o", op) for (t, op) in extra]
    # stable sort by time; later times act further left
    items = sorted(enumerate(items), key=lambda it: (it[1][0], it[0]))
    e, v = np.linalg.eigh(H0)
    e0 = e.min()

    def prop(dt):
        return (v * np.exp(-dt * (e - e0))) @ v.T

    M = np.eye(f.dim)
    t_prev = 0.0
    for _, (t, kind, payload) in items:
        M = prop(t - t_prev) @ M
        if kind == "v":
            x, s = payload
            op = np.diag(np.exp(gamma * s * (np.diag(f.n[f.mode(x, 0)]) - np.diag(f.n[f.mode(x, 1)]))))
        else:
            op = payload
        M = op @ M
        t_prev = t
    M = prop(beta - t_prev) @ M
    return float(np.trace(M))


def trace_ratio(f: Fock, H0: np.ndarray, beta: float, gamma: float, verts) -> float:
    """Z_n({s_i, tau_i}) / Z_0 (Eqs. (Zn) and (Zn_div_Z0))."""
    return vertex_product(f, H0, beta, gamma, verts) / vertex_product(f, H0, beta, gamma, [])


def greens_with_vertices(f: Fock, H0, beta, gamma, verts, x, y, spin, tau) -> float:
    """<T c_x(tau) c_y^dagger(0)> in the field of the auxiliary spins, 0 < tau."""
    cy_dag = f.c[f.mode(y, spin)].T
    cx = f.c[f.mode(x, spin)]
    num = vertex_product(f, H0, beta, gamma, verts, extra=[(0.0, cy_dag), (tau, cx)])
    den = vertex_product(f, H0, beta, gamma, verts)
    return num / den
