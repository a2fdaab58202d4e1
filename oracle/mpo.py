"""Generic matrix-product operator of the active-space Hamiltonian, built from
its list of second-quantised terms.  TEST INFRASTRUCTURE ONLY (see
``oracle/__init__.py``).

The Hamiltonian is the normal-ordered active-space operator (Sec. II.A, with
the Cholesky factorisation (pq|rs) = sum_Q B^Q_pq B^Q_rs)

    H = sum_pq h_pq sum_s a+_{ps} a_{qs}
      + 1/2 sum_pqrs (pq|rs) sum_{s,t} a+_{ps} a+_{rt} a_{st} a_{qs},

written out term by term.  Sites are spatial orbitals with the 4 states
s = n_alpha + 2 n_beta; the Jordan-Wigner order is interleaved (0a, 0b, 1a,
1b, ...), so a ladder operator on mode j carries the parity of every occupied
mode before it: F on each earlier site, and on its own site the parity of the
alpha mode when j is the beta mode (``site_ops``).

This MPO shares nothing with the product library's MPO (which is built from
hand-designed channel families with Cholesky density channels).  Here every
term is a path through an automaton:

* each term is first brought to site order (a stable sort of its ladder
  operators by (site, spin); every swap passes two distinct modes, so it flips
  the sign), and terms that become the same operator string are summed;
* at a cut c the term is *left-carried* while its ladder operators left of c
  are fewer than those right of it (or as many, for c <= L/2): the channel is
  labelled by the operator string already placed on the left, and the
  coefficient is still pending;
* afterwards it is *right-carried*: the channel is labelled by the operator
  string still to come on the right, and the coefficient has been applied;
* the switch happens once, at the site where the term leaves the left-carried
  regime; that site's MPO entry carries the coefficient.  Chains before and
  after the switch are shared by all terms with the same label.

The sum over paths from the left boundary channel ``I`` to the right boundary
channel ``D`` is then exactly sum_t c_t (term t): every left-carried label has
one incoming chain (its own prefix) and every right-carried label one outgoing
chain (its own suffix), so a path through a switch entry (alpha, beta, op) is
prefix(alpha) (x) op (x) suffix(beta) with the summed coefficients of the terms
that share all three.

The constant e_core is not part of the MPO (H_eff excludes it, as in the
product library).

Pins (``tests/test_oracle_blocks.py``): the MPO contracted to a dense 4^L x 4^L
matrix equals the brute-force Fock-space H of ``oracle.fock`` (interleaved
order) for L <= 4 at several integral sets, including one-body-only and
two-body-only Hamiltonians.
"""
from __future__ import annotations

import numpy as np

# ------------------------------------------------------------ site operators --
# Site states s = n_alpha + 2 n_beta (bit 0: alpha mode, bit 1: beta mode).
_F = np.diag([1.0, -1.0, -1.0, 1.0])


def _ladder(mode: int, create: bool) -> np.ndarray:
    """<s_out|a(+)_mode|s_in> on one site: the mode's occupation flips and the
    sign is the parity of the occupied modes of the site ordered before it."""
    M = np.zeros((4, 4))
    for s in range(4):
        occ = (s >> mode) & 1
        if occ == (1 if create else 0):
            continue
        below = bin(s & ((1 << mode) - 1)).count("1")
        M[s ^ (1 << mode), s] = -1.0 if below & 1 else 1.0
    return M


def site_ops():
    """Dict of the site matrices: ('c', spin) creators, ('a', spin) annihilators, 'F' parity."""
    out = {"F": _F.copy()}
    for spin in (0, 1):
        out[("c", spin)] = _ladder(spin, True)
        out[("a", spin)] = _ladder(spin, False)
    return out


_OPS = site_ops()


def local_matrix(local_key) -> np.ndarray:
    """Product, in operator order, of the ladder operators (spin, dagger) of one site."""
    M = np.eye(4)
    for spin, dag in local_key:
        M = M @ _OPS[("c" if dag else "a", spin)]
    return M


def _charge(spin, dag):
    dn = 1 if dag else -1
    return (dn, dn if spin == 0 else -dn)


# --------------------------------------------------------------------- terms --
def hamiltonian_terms(h, B):
    """Normal-ordered terms of H - e_core, in site order, equal strings summed.

    Returns a dict: tuple of (site, spin, dagger) in site order -> coefficient.
    """
    h = np.asarray(h, dtype=float)
    B = np.asarray(B, dtype=float)
    n = h.shape[0]
    g = np.einsum("Qpq,Qrs->pqrs", B, B) if B.size else np.zeros((n, n, n, n))
    terms = {}

    def add(coef, ops):
        if coef == 0.0:
            return
        # stable sort by (site, spin): each swap exchanges two distinct modes
        key = [(o[0], o[1]) for o in ops]
        order = sorted(range(len(ops)), key=lambda i: key[i])
        inv = 0
        for i in range(len(order)):
            for j in range(i + 1, len(order)):
                if order[i] > order[j]:
                    inv += 1
        srt = tuple(ops[i] for i in order)
        c = -coef if inv & 1 else coef
        terms[srt] = terms.get(srt, 0.0) + c

    for p in range(n):
        for q in range(n):
            for s in (0, 1):
                add(h[p, q], [(p, s, 1), (q, s, 0)])
    for p in range(n):
        for q in range(n):
            for r in range(n):
                for t in range(n):
                    c = 0.5 * g[p, q, r, t]
                    if c == 0.0:
                        continue
                    for s1 in (0, 1):
                        for s2 in (0, 1):
                            if (p, s1) == (r, s2) or (t, s2) == (q, s1):
                                continue  # a+ a+ (or a a) on one mode vanishes
                            add(c, [(p, s1, 1), (r, s2, 1), (t, s2, 0), (q, s1, 0)])
    return {k: v for k, v in terms.items() if v != 0.0}


# ----------------------------------------------------------------------- MPO --
class MPO:
    """W[x]: dict (a, b, opkey) -> coefficient for site x (channel a at cut x,
    channel b at cut x+1).  opkey = (local_key, parity): the site matrix is
    local_matrix(local_key) @ F^parity.  dq[c][a] = (dN, d2Sz) of the left part
    of channel a at cut c.  Cut 0 holds the single channel 'I', cut L the
    single channel 'D'."""

    def __init__(self, L):
        self.L = L
        self.labels = [dict() for _ in range(L + 1)]
        self.dq = [[] for _ in range(L + 1)]
        self.W = [dict() for _ in range(L)]

    def chan(self, c, label, dq):
        d = self.labels[c]
        i = d.get(label)
        if i is None:
            i = len(d)
            d[label] = i
            self.dq[c].append(dq)
        return i

    def dims(self):
        return [len(x) for x in self.labels]

    @staticmethod
    def op_matrix(opkey):
        local_key, parity = opkey
        M = local_matrix(local_key)
        return M @ _F if parity else M


def build_mpo(h, B):
    """The automaton MPO of H - e_core (see the module docstring)."""
    n = np.asarray(h).shape[0]
    L = n
    mpo = MPO(L)
    half = L // 2
    terms = hamiltonian_terms(h, B)
    left_done = set()   # (cut, label) whose incoming chain exists
    right_done = set()  # (cut, label) whose outgoing chain exists
    for ops, coef in terms.items():
        m = len(ops)
        # ladder operators grouped by site (already in site order)
        sites, locs = [], []
        for (x, spin, dag) in ops:
            if sites and sites[-1] == x:
                locs[-1].append((spin, dag))
            else:
                sites.append(x)
                locs.append([(spin, dag)])
        locs = [tuple(l) for l in locs]
        counts = [len(l) for l in locs]
        charges = []
        for l in locs:
            dn = sum(_charge(s, d)[0] for s, d in l)
            ds = sum(_charge(s, d)[1] for s, d in l)
            charges.append((dn, ds))

        def nl(c):
            return sum(k for x, k in zip(sites, counts) if x < c)

        def left_carried(c):
            a, b = nl(c), m - nl(c)
            return a < b or (a == b and c <= half)

        sw = 0
        while sw + 1 <= L - 1 and left_carried(sw + 1):
            sw += 1

        def site_op(x):
            after = sum(k for y, k in zip(sites, counts) if y > x)
            loc = ()
            for y, l in zip(sites, locs):
                if y == x:
                    loc = l
            return (loc, after & 1)

        def left_label(c):
            pre = tuple((y, l) for y, l in zip(sites, locs) if y < c)
            if not pre:
                return "I", (0, 0)
            dn = sum(q[0] for y, q in zip(sites, charges) if y < c)
            ds = sum(q[1] for y, q in zip(sites, charges) if y < c)
            return ("L",) + pre, (dn, ds)

        def right_label(c):
            suf = tuple((y, l) for y, l in zip(sites, locs) if y >= c)
            if not suf:
                return "D", (0, 0)
            dn = sum(q[0] for y, q in zip(sites, charges) if y >= c)
            ds = sum(q[1] for y, q in zip(sites, charges) if y >= c)
            return ("R",) + suf, (-dn, -ds)

        # left chain into the switch cut (shared by every term with this prefix)
        lab, dq = left_label(sw)
        a_sw = mpo.chan(sw, lab, dq)
        c = sw
        while c > 0 and (c, lab) not in left_done:
            left_done.add((c, lab))
            plab, pdq = left_label(c - 1)
            a = mpo.chan(c - 1, plab, pdq)
            b = mpo.chan(c, lab, dq)
            mpo.W[c - 1][(a, b, site_op(c - 1))] = 1.0
            c, lab, dq = c - 1, plab, pdq
        # the switch entry carries the coefficient
        rlab, rdq = right_label(sw + 1)
        b_sw = mpo.chan(sw + 1, rlab, rdq)
        key = (a_sw, b_sw, site_op(sw))
        mpo.W[sw][key] = mpo.W[sw].get(key, 0.0) + coef
        # right chain out of the switch cut (shared by every term with this suffix)
        c, lab, dq = sw + 1, rlab, rdq
        while c < L and (c, lab) not in right_done:
            right_done.add((c, lab))
            nlab, ndq = right_label(c + 1)
            a = mpo.chan(c, lab, dq)
            b = mpo.chan(c + 1, nlab, ndq)
            mpo.W[c][(a, b, site_op(c))] = 1.0
            c, lab, dq = c + 1, nlab, ndq
    # boundary channels exist even for an empty Hamiltonian
    mpo.chan(0, "I", (0, 0))
    mpo.chan(L, "D", (0, 0))
    return mpo


def site_tensor(mpo: MPO, x: int) -> np.ndarray:
    """Dense W_x[a, b, s, s'] (for tiny L)."""
    Da, Db = len(mpo.labels[x]), len(mpo.labels[x + 1])
    W = np.zeros((Da, Db, 4, 4))
    for (a, b, opkey), c in mpo.W[x].items():
        W[a, b] += c * MPO.op_matrix(opkey)
    return W


def dense(mpo: MPO) -> np.ndarray:
    """The MPO contracted to a dense 4^L x 4^L matrix in the site-product basis
    (index sum_p s_p 4^(L-1-p)); tiny L only."""
    L = mpo.L
    I0 = mpo.labels[0]["I"]
    D = mpo.labels[L]["D"]
    # T[a][out, in] over the sites so far
    W0 = site_tensor(mpo, 0)
    T = W0[I0]  # [b, s, s']
    for x in range(1, L):
        W = site_tensor(mpo, x)
        T = np.einsum("aij,abkl->bikjl", T, W)
        nb, d1, d2, d3, d4 = T.shape
        T = T.reshape(nb, d1 * d2, d3 * d4)
    return T[D]
