"""Determinant-space FCI for H = sum h_pq E_pq + 1/2 sum (pq|rs)(E_pq E_rs - d_qr E_ps).

Definitions (the active-space Hamiltonian of Sec. II.A with the Cholesky
factorisation (pq|rs) = sum_Q B^Q_pq B^Q_rs):

* E_pq = sum_sigma a+_{p sigma} a_{q sigma}.
* Determinants |I_a I_b> = (prod_{p in I_a} a+_{p alpha}) (prod_{p in I_b} a+_{p beta}) |0>,
  creators in ascending orbital order, all alpha before all beta.
* Strings are ranked colexicographically, addr = sum_i C(o_i, i + 1) over the
  sorted occupied orbitals (Sec. III, device CI addressing).
* The CI vector is a matrix c[I_a, I_b].

Pins: ``tests/test_oracle_fci.py`` (brute-force Fock space, free fermions,
Hubbard dimer, Hermiticity, S^2 integrality, RDM traces, Euler identity, finite
differences of the energy; transition RDMs against products of brute-force
Fock-space one-body operators and a hand-worked two-orbital case).
"""
from __future__ import annotations

from itertools import combinations
from math import comb

import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------- strings --
def colex_address(occ) -> int:
    """addr = sum_i C(o_i, i+1) over sorted occupied orbitals o_0 < o_1 < ..."""
    return sum(comb(o, i + 1) for i, o in enumerate(sorted(occ)))


def strings(n: int, k: int) -> np.ndarray:
    """All n-bit strings with k bits set, as int64 bitmasks, in colex order."""
    out = [0] * comb(n, k)
    for occ in combinations(range(n), k):
        out[colex_address(occ)] = sum(1 << o for o in occ)
    return np.array(out, dtype=np.int64)


def _popcount(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.int64)
    c = np.zeros_like(x)
    while np.any(x):
        c += x & 1
        x = x >> 1
    return c


def string_excitation(n: int, strs: np.ndarray):
    """e[p][q]: sparse matrix of E_pq restricted to one spin, on `strs`.

    E_pq |J> = sign |I>: a_q removes q with sign (-1)^(#occupied below q), then
    a+_p inserts p with sign (-1)^(#occupied below p in the new string).
    """
    index = {int(s): i for i, s in enumerate(strs)}
    N = len(strs)
    e = [[None] * n for _ in range(n)]
    for p in range(n):
        for q in range(n):
            rows, cols, vals = [], [], []
            for j, s in enumerate(strs):
                s = int(s)
                if not (s >> q) & 1:
                    continue
                s1 = s & ~(1 << q)
                sgn = -1 if bin(s1 & ((1 << q) - 1)).count("1") & 1 else 1
                if (s1 >> p) & 1:
                    continue
                s2 = s1 | (1 << p)
                if bin(s1 & ((1 << p) - 1)).count("1") & 1:
                    sgn = -sgn
                rows.append(index[s2])
                cols.append(j)
                vals.append(float(sgn))
            e[p][q] = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    return e


class DetSpace:
    """Determinant space of n orbitals with n_alpha, n_beta electrons."""

    def __init__(self, n: int, n_alpha: int, n_beta: int):
        self.n, self.na, self.nb = n, n_alpha, n_beta
        self.sa = strings(n, n_alpha)
        self.sb = strings(n, n_beta)
        self.ea = string_excitation(n, self.sa)
        self.eb = self.ea if n_alpha == n_beta else string_excitation(n, self.sb)
        self.shape = (len(self.sa), len(self.sb))
        self.size = self.shape[0] * self.shape[1]

    def occ(self):
        """Occupation matrices (n_str x n) for alpha and beta strings."""
        oa = ((self.sa[:, None] >> np.arange(self.n)) & 1).astype(float)
        ob = ((self.sb[:, None] >> np.arange(self.n)) & 1).astype(float)
        return oa, ob

    def apply_E(self, p: int, q: int, C: np.ndarray) -> np.ndarray:
        """E_pq C (E^beta carries no alpha parity: it is an even operator)."""
        return self.ea[p][q] @ C + (self.eb[p][q] @ C.T).T


# ------------------------------------------------------------ Hamiltonian --
def eri(B: np.ndarray) -> np.ndarray:
    """(pq|rs) = sum_Q B^Q_pq B^Q_rs (Sec. II.A factorisation)."""
    return np.einsum("Qpq,Qrs->pqrs", B, B)


def one_body_shift(h: np.ndarray, g: np.ndarray) -> np.ndarray:
    """t_pq = h_pq - 1/2 sum_r (pr|rq), so H = sum t E + 1/2 sum g E E."""
    return h - 0.5 * np.einsum("prrq->pq", g)


def sigma(space: DetSpace, h, g, C, e_core: float = 0.0) -> np.ndarray:
    """Knowles-Handy sigma: D_rs = E_rs C, G_pq = sum_rs (pq|rs) D_rs,
    sigma = e_core C + sum t_pq E_pq C + 1/2 sum_pq E_pq G_pq."""
    n = space.n
    C = C.reshape(space.shape)
    t = one_body_shift(h, g)
    D = np.empty((n * n,) + space.shape)
    for r in range(n):
        for s in range(n):
            D[r * n + s] = space.apply_E(r, s, C)
    G = (g.reshape(n * n, n * n) @ D.reshape(n * n, -1)).reshape(D.shape)
    out = e_core * C + np.tensordot(t.reshape(-1), D, axes=(0, 0))
    for p in range(n):
        for q in range(n):
            out += 0.5 * space.apply_E(p, q, G[p * n + q])
    return out


def diagonal(space: DetSpace, h, g, e_core: float = 0.0) -> np.ndarray:
    """<I|H|I> = e_core + sum_p t_pp n_p + 1/2 sum_pr (pp|rr) n_p n_r
    + 1/2 sum_{r != s} (sr|rs) sum_sigma n_{s sigma}(1 - n_{r sigma})."""
    oa, ob = space.occ()
    t = one_body_shift(h, g)
    J = np.einsum("pprr->pr", g)
    K = np.einsum("srrs->sr", g).copy()
    np.fill_diagonal(K, 0.0)
    na = oa[:, None, :]
    nb = ob[None, :, :]
    ntot = na + nb
    d = e_core + ntot @ np.diag(t)
    d += 0.5 * np.einsum("abp,pr,abr->ab", ntot, J, ntot)
    for occ in (oa, ob):
        x = occ @ K @ (1.0 - occ).T  # sum_{s,r} n_s K_sr (1 - n_r)
        d += 0.5 * (np.diag(x)[:, None] if occ is oa else np.diag(x)[None, :])
    return d


def dense_hamiltonian(space: DetSpace, h, g, e_core: float = 0.0) -> np.ndarray:
    """Dense H by applying sigma to unit vectors (small spaces only)."""
    N = space.size
    H = np.empty((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        H[:, j] = sigma(space, h, g, e, e_core).reshape(-1)
    return H


# ------------------------------------------------------------- eigensolve --
def davidson(apply, diag, nroots: int, tol: float = 1e-9, max_iter: int = 300,
             max_sub: int = 40, seed: int = 0):
    """Plain block Davidson with the diagonal preconditioner (lowest roots).

    Converged when every root has ||H x - theta x|| <= tol.  Cross-checked in
    the tests against dense eigh and scipy's eigsh.
    """
    N = diag.size
    rng = np.random.default_rng(seed)
    order = np.argsort(diag)
    V = np.zeros((N, nroots))
    for i in range(nroots):
        V[order[i], i] = 1.0
    V += 1e-3 * rng.standard_normal(V.shape)
    V, _ = np.linalg.qr(V)
    W = np.column_stack([apply(V[:, i]) for i in range(V.shape[1])])
    for _ in range(max_iter):
        Hs = V.T @ W
        Hs = 0.5 * (Hs + Hs.T)
        th, y = np.linalg.eigh(Hs)
        th, y = th[:nroots], y[:, :nroots]
        X = V @ y
        R = W @ y - X * th
        rn = np.linalg.norm(R, axis=0)
        if np.all(rn <= tol):
            return th, X
        if V.shape[1] + nroots > max_sub:
            V, W = X.copy(), W @ y
        new = []
        for i in range(nroots):
            if rn[i] <= tol:
                continue
            den = th[i] - diag
            den[np.abs(den) < 1e-8] = 1e-8
            t = R[:, i] / den
            for _ in range(2):
                t -= V @ (V.T @ t)
                for u in new:
                    t -= u * (u @ t)
            nt = np.linalg.norm(t)
            if nt > 1e-12:
                new.append(t / nt)
        if not new:
            return th, X
        Nw = np.column_stack(new)
        V = np.column_stack([V, Nw])
        W = np.column_stack([W] + [apply(u) for u in new])
    raise RuntimeError("oracle davidson did not converge")


def solve(n, n_alpha, n_beta, h, B, nroots=1, e_core=0.0, tol=1e-9, dense_limit=3000):
    """Lowest `nroots` energies and CI vectors (dense eigh for small spaces)."""
    space = DetSpace(n, n_alpha, n_beta)
    g = eri(B)
    if space.size <= dense_limit:
        H = dense_hamiltonian(space, h, g, e_core)
        w, v = np.linalg.eigh(H)
        return w[:nroots], [v[:, i].reshape(space.shape) for i in range(nroots)], space
    d = diagonal(space, h, g, e_core).reshape(-1)
    th, X = davidson(lambda x: sigma(space, h, g, x, e_core).reshape(-1), d, nroots, tol)
    return th, [X[:, i].reshape(space.shape) for i in range(nroots)], space


# -------------------------------------------------------------------- RDMs --
def rdm12(space: DetSpace, C: np.ndarray):
    """gamma_pq = <E_pq>, Gamma'_pqrs = <E_pq E_rs> - d_qr gamma_ps."""
    n = space.n
    C = C.reshape(space.shape)
    D = np.empty((n, n) + space.shape)
    for r in range(n):
        for s in range(n):
            D[r, s] = space.apply_E(r, s, C)
    gamma = np.einsum("ab,pqab->pq", C, D)
    # <E_pq E_rs> = <E_qp c | E_rs c>
    EE = np.einsum("qpab,rsab->pqrs", D, D)
    Gp = EE - np.einsum("qr,ps->pqrs", np.eye(n), gamma)
    return gamma, Gp


def trdm12(space: DetSpace, Cbra: np.ndarray, Cket: np.ndarray):
    """Transition RDMs by nested application, straight from the definitions:
    gamma_pq = <bra|E_pq|ket>, Gamma'_pqrs = <bra|E_pq E_rs|ket> - d_qr gamma_ps
    (E_rs applied to the ket first, then E_pq; no adjoint identity used)."""
    n = space.n
    Cb = Cbra.reshape(space.shape)
    Ck = Cket.reshape(space.shape)
    gamma = np.empty((n, n))
    EE = np.empty((n, n, n, n))
    for r in range(n):
        for s in range(n):
            D = space.apply_E(r, s, Ck)
            gamma[r, s] = np.sum(Cb * D)
            for p in range(n):
                for q in range(n):
                    EE[p, q, r, s] = np.sum(Cb * space.apply_E(p, q, D))
    Gp = EE - np.einsum("qr,ps->pqrs", np.eye(n), gamma)
    return gamma, Gp


def rdm3(space: DetSpace, Cbra: np.ndarray, Cket: np.ndarray, picks=None):
    """Transition three-body density <bra|E_pq E_rs E_tu|ket> by nested
    application (E_tu first).  picks: optional list of (p, q, r, s, t, u) to
    evaluate one by one (returns a list); else the full n^6 array."""
    n = space.n
    Cb = Cbra.reshape(space.shape)
    Ck = Cket.reshape(space.shape)
    if picks is not None:
        return [float(np.sum(Cb * space.apply_E(p, q, space.apply_E(r, s, space.apply_E(t, u, Ck)))))
                for p, q, r, s, t, u in picks]
    out = np.empty((n,) * 6)
    for t in range(n):
        for u in range(n):
            D1 = space.apply_E(t, u, Ck)
            for r in range(n):
                for s in range(n):
                    D2 = space.apply_E(r, s, D1)
                    for p in range(n):
                        for q in range(n):
                            out[p, q, r, s, t, u] = np.sum(Cb * space.apply_E(p, q, D2))
    return out


def apply_v(space: DetSpace, B: np.ndarray, C: np.ndarray) -> np.ndarray:
    """V C, V = 1/2 sum_pqrs (pq|rs) E_pq E_rs, term by term from the definition."""
    n = space.n
    g = eri(B)
    C = C.reshape(space.shape)
    out = np.zeros(space.shape)
    for r in range(n):
        for s in range(n):
            D = space.apply_E(r, s, C)
            for p in range(n):
                for q in range(n):
                    if g[p, q, r, s] != 0.0:
                        out += 0.5 * g[p, q, r, s] * space.apply_E(p, q, D)
    return out


def energy_from_rdm(h, B, gamma, Gp, e_core=0.0):
    g = eri(B)
    return e_core + np.einsum("pq,pq->", h, gamma) + 0.5 * np.einsum("pqrs,pqrs->", g, Gp)


def integral_gradients(B, gamma, Gp):
    """dE/dh_pq = gamma_pq; dE/dB^Q_pq = sum_rs Gamma'_pqrs B^Q_rs (entries independent)."""
    return gamma.copy(), np.einsum("pqrs,Qrs->Qpq", Gp, B)


# ---------------------------------------------------------------------- S^2 --
def _apply_ladder(bits: int, so: int, create: bool):
    """Ladder op on spin-orbital `so` of a determinant bitmask (alpha-first order)."""
    occ = (bits >> so) & 1
    if create == bool(occ):
        return None, 0
    sgn = -1 if bin(bits & ((1 << so) - 1)).count("1") & 1 else 1
    return bits ^ (1 << so), sgn


def s_squared(space: DetSpace, C: np.ndarray) -> float:
    """<S^2> = ||S_+ c||^2 + S_z (S_z + 1) with S_+ = sum_p a+_{p alpha} a_{p beta}."""
    n = space.n
    C = C.reshape(space.shape)
    if space.nb == 0:
        sz = 0.5 * (space.na - space.nb)
        return sz * (sz + 1) * float(np.sum(C * C))
    ta = strings(n, space.na + 1)
    tb = strings(n, space.nb - 1)
    ia = {int(s): i for i, s in enumerate(ta)}
    ib = {int(s): i for i, s in enumerate(tb)}
    out = np.zeros((len(ta), len(tb)))
    for i, sa in enumerate(space.sa):
        for j, sb in enumerate(space.sb):
            bits = int(sa) | (int(sb) << n)
            for p in range(n):
                b1, s1 = _apply_ladder(bits, n + p, False)
                if b1 is None:
                    continue
                b2, s2 = _apply_ladder(b1, p, True)
                if b2 is None:
                    continue
                out[ia[b2 & ((1 << n) - 1)], ib[b2 >> n]] += s1 * s2 * C[i, j]
    sz = 0.5 * (space.na - space.nb)
    return float(np.sum(out * out)) + sz * (sz + 1) * float(np.sum(C * C))


def _ladder_matrix(n: int, src: np.ndarray, dst: np.ndarray, p: int, create: bool):
    """One spin's a+_p (create) or a_p on strings src -> dst, with the sign
    (-1)^(#occupied orbitals below p) of moving the operator into place."""
    index = {int(s): i for i, s in enumerate(dst)}
    rows, cols, vals = [], [], []
    for j, s in enumerate(src):
        s = int(s)
        occ = (s >> p) & 1
        if occ == int(create):
            continue
        t = s ^ (1 << p)
        sgn = -1.0 if bin(s & ((1 << p) - 1)).count("1") & 1 else 1.0
        rows.append(index[t])
        cols.append(j)
        vals.append(sgn)
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(dst), len(src)))


def s_squared_sparse(space: DetSpace, C: np.ndarray) -> float:
    """<S^2> = ||S_+ c||^2 + S_z (S_z + 1) with S_+ = sum_p a+_{p alpha} a_{p beta},
    applied as sparse string operators: (S_+ C)[I'_a, I'_b] = sum_p
    cre_p[I'_a, I_a] C[I_a, I_b] ann_p[I'_b, I_b] (up to the global sign
    (-1)^(n_alpha) of taking a_{p beta} past the alpha string, which the norm drops)."""
    n = space.n
    C = C.reshape(space.shape)
    sz = 0.5 * (space.na - space.nb)
    base = sz * (sz + 1) * float(np.sum(C * C))
    if space.nb == 0 or space.na == n:
        return base
    ta = strings(n, space.na + 1)
    tb = strings(n, space.nb - 1)
    out = np.zeros((len(ta), len(tb)))
    for p in range(n):
        cre = _ladder_matrix(n, space.sa, ta, p, True)
        ann = _ladder_matrix(n, space.sb, tb, p, False)
        out += cre @ (ann @ C.T).T
    return float(np.sum(out * out)) + base

