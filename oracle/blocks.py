"""Block-sparse environments, two-site sigma and H_eff diagonal on the oracle's
own MPO (``oracle.mpo``).  TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Definitions (the DMRG decimation step of Fig. 2 / Sec. II.H; the matrix-free
two-site H_eff of the sweep):

* Bond sectors are (N, 2S_z) labels of the left part of a cut; a site tensor
  A[a, s, b] is nonzero only for q_b = q_a + q_s (site states s = n_alpha +
  2 n_beta carry q_s = (0,0), (1,1), (1,-1), (2,0)).
* Left environment at cut c, channel alpha of the MPO cut c:
      L_c[alpha]_{a a'} = <a| O^left_alpha |a'>,
  with |a> = sum A_0 ... A_{c-1} the left-block states.  Recursion over site x:
      L_{x+1}[beta] = sum_{alpha, s, s'} W_x[alpha, beta]_{s s'} A_s^T L_x[alpha] A_{s'}.
* Right environment at cut c (sites c..L-1):
      R_x[alpha] = sum_{beta, s, s'} W_x[alpha, beta]_{s s'} A_s R_{x+1}[beta] A_{s'}^T.
* Two-site sigma on sites (k, k+1):
      sigma[a s1 s2 b] = sum L_k[alpha]_{a a'} W_k[alpha,beta]_{s1 s1'}
                         W_{k+1}[beta,gamma]_{s2 s2'} R_{k+2}[gamma]_{b b'} psi[a' s1' s2' b'],
  evaluated as sum_beta (sum_alpha ...) psi (sum_gamma ...)^T: the left sums
  X_{beta,O} = sum_alpha c L_k[alpha] per site operator O of W_k, the right sums
  Y_{beta,O'} = sum_gamma c R_{k+2}[gamma] per site operator O' of W_{k+1}.
  The Jordan-Wigner signs live in the site operators, so these are plain
  tensor contractions.
* The diagonal of H_eff is the same sum restricted to a = a', s = s', b = b'.

A channel alpha with left-part charge dq maps ket sector q' to bra sector
q' + dq, so the blocks of all channels with one dq share one block list; the
environments store, per dq class and block, one array [channel, bra, ket].
Environment updates mix the channels of a class with one matrix product per
block (a library product over the stacked channels) and apply the site
tensors to all mixed channels of a block at once.

Pins (``tests/test_oracle_blocks.py``): sigma equals the projected FCI sigma
P^T H P psi of ``oracle.embed`` (determinant space, no MPO, no environments)
for random MPS at exact and truncated bonds, every step k, including ragged
sectors; the diagonal equals the diagonal of the dense P^T H P built from unit
vectors; H_eff is symmetric.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mpo import MPO

SITE_QN = ((0, 0), (1, 1), (1, -1), (2, 0))


def _add(q, d):
    return (q[0] + d[0], q[1] + d[1])


def _sub(q, d):
    return (q[0] - d[0], q[1] - d[1])


def _qdiff(a, b):
    return (a[0] - b[0], a[1] - b[1])


class Bond:
    def __init__(self, sectors):
        self.sec = [tuple(int(v) for v in s) for s in sectors]
        self.idx = {(s[0], s[1]): i for i, s in enumerate(self.sec)}

    def q(self, i):
        return (self.sec[i][0], self.sec[i][1])

    def dim(self, i):
        return self.sec[i][2]

    def find(self, q):
        return self.idx.get((q[0], q[1]))

    def __len__(self):
        return len(self.sec)


# ------------------------------------------------------------- slab layout --
def slab_blocks(bond_l: Bond, bond_r: Bond, phys_qn):
    """Yield (l, p, r, start, width, col0): block (left sector l, physical p,
    right sector r) of a slab-layout vector: for each left sector a row-major
    m_l x width slab whose columns are the blocks of the physical states in
    order whose right sector exists."""
    start = 0
    for l in range(len(bond_l)):
        ql = bond_l.q(l)
        cols = []
        for p, dq in enumerate(phys_qn):
            r = bond_r.find(_add(ql, dq))
            if r is not None:
                cols.append((p, r))
        width = sum(bond_r.dim(r) for _, r in cols)
        c0 = 0
        for p, r in cols:
            yield l, p, r, start, width, c0
            c0 += bond_r.dim(r)
        start += bond_l.dim(l) * width


def unpack(bond_l: Bond, bond_r: Bond, phys_qn, flat):
    """Slab-layout vector -> dict (l, p, r) -> m_l x m_r array."""
    out = {}
    for l, p, r, start, width, c0 in slab_blocks(bond_l, bond_r, phys_qn):
        ml, mr = bond_l.dim(l), bond_r.dim(r)
        slab = np.asarray(flat[start:start + ml * width]).reshape(ml, width)
        out[(l, p, r)] = slab[:, c0:c0 + mr]
    return out


def pack(bond_l: Bond, bond_r: Bond, phys_qn, blocks):
    """dict (l, p, r) -> block, back to the slab-layout vector (missing blocks are zero)."""
    size = 0
    for l, p, r, start, width, c0 in slab_blocks(bond_l, bond_r, phys_qn):
        size = max(size, start + bond_l.dim(l) * width)
    out = np.zeros(size)
    for l, p, r, start, width, c0 in slab_blocks(bond_l, bond_r, phys_qn):
        b = blocks.get((l, p, r))
        if b is None:
            continue
        ml, mr = bond_l.dim(l), bond_r.dim(r)
        v = out[start:start + ml * width].reshape(ml, width)
        v[:, c0:c0 + mr] = b
    return out


def twosite_qn():
    return [_add(SITE_QN[a], SITE_QN[b]) for a in range(4) for b in range(4)]


# -------------------------------------------------------------- environments --
class Env:
    """Environment at one cut: per dq class, channels and blocks [n_ch, bra, ket]."""

    def __init__(self, bond: Bond, dq):
        self.bond = bond
        self.dq = list(dq)  # per channel of the MPO cut
        self.classes = {}
        for ch, d in enumerate(self.dq):
            cl = self.classes.setdefault(d, {"chans": [], "blocks": {}})
            cl["chans"].append(ch)
        for cl in self.classes.values():
            cl["slot"] = {ch: i for i, ch in enumerate(cl["chans"])}

    def block(self, d, bra, ket):
        """[n_ch, m_bra, m_ket] array of class d (allocated as zeros on first use)."""
        cl = self.classes[d]
        arr = cl["blocks"].get((bra, ket))
        if arr is None:
            arr = np.zeros((len(cl["chans"]), self.bond.dim(bra), self.bond.dim(ket)))
            cl["blocks"][(bra, ket)] = arr
        return arr

    def channel(self, ch):
        """dict (bra, ket) -> block of one channel (views)."""
        d = self.dq[ch]
        cl = self.classes[d]
        i = cl["slot"][ch]
        return {k: v[i] for k, v in cl["blocks"].items()}


def left_boundary(mpo: MPO, bond0: Bond):
    e = Env(bond0, mpo.dq[0])
    I = mpo.labels[0]["I"]
    e.block((0, 0), 0, 0)[e.classes[(0, 0)]["slot"][I]] = 1.0
    return e


def right_boundary(mpo: MPO, bondL: Bond):
    e = Env(bondL, mpo.dq[mpo.L])
    D = mpo.labels[mpo.L]["D"]
    e.block((0, 0), 0, 0)[e.classes[(0, 0)]["slot"][D]] = 1.0
    return e


def _groups(entries, by_left):
    """Entries (a, b, opkey) -> c grouped by (output channel, opkey): list of (src, c).
    by_left: the output channel is b (left env / sigma left side), else a."""
    g = {}
    for (a, b, opkey), c in entries.items():
        if c == 0.0:
            continue
        key = (b, opkey) if by_left else (a, opkey)
        g.setdefault(key, []).append((a if by_left else b, c))
    return g


def _mix_rows(env: Env, groups, dq_src):
    """Rows (output channel, opkey) grouped by their source class, with the
    sparse mixing matrix C[row, source slot] of each class."""
    per_class = {}
    for key, srcs in groups.items():
        d = dq_src[srcs[0][0]]
        for s, _ in srcs:
            assert dq_src[s] == d, "sources of one mixed row in different classes"
        per_class.setdefault(d, []).append(key)
    out = {}
    for d, rows in per_class.items():
        if d not in env.classes:
            continue
        cl = env.classes[d]
        ri, ci, vals = [], [], []
        for i, key in enumerate(rows):
            for s, c in groups[key]:
                ri.append(i)
                ci.append(cl["slot"][s])
                vals.append(c)
        C = sp.csr_matrix((vals, (ri, ci)), shape=(len(rows), len(cl["chans"])))
        out[d] = (rows, C)
    return out


def _scatter_into(out_arr, slots, weights, Z):
    """out_arr[slot_j] += weights[j] * Z[j] (slots may repeat)."""
    n_out = out_arr.shape[0]
    S = sp.csr_matrix((weights, (slots, np.arange(len(slots)))), shape=(n_out, len(slots)))
    out_arr += (S @ Z.reshape(len(slots), -1)).reshape(out_arr.shape)


def update_left(env: Env, A: dict, bond_r: Bond, mpo: MPO, x: int, flops=None):
    """L_{x+1} from L_x and the site tensor A (dict (l, s, r) -> block)."""
    out = Env(bond_r, mpo.dq[x + 1])
    groups = _groups(mpo.W[x], by_left=True)
    for d, (rows, C) in _mix_rows(env, groups, mpo.dq[x]).items():
        ops = np.array([MPO.op_matrix(k[1]) for k in rows])  # [row, s, s']
        outch = np.array([k[0] for k in rows])
        for (l, lp), data in env.classes[d]["blocks"].items():
            n_ch, ml, mlp = data.shape
            X = (C @ data.reshape(n_ch, -1)).reshape(len(rows), ml, mlp)
            for s in range(4):
                r = bond_r.find(_add(env.bond.q(l), SITE_QN[s]))
                if r is None or (l, s, r) not in A:
                    continue
                As = A[(l, s, r)]
                for t in range(4):
                    w = ops[:, s, t]
                    sel = np.nonzero(w)[0]
                    if sel.size == 0:
                        continue
                    rp = bond_r.find(_add(env.bond.q(lp), SITE_QN[t]))
                    if rp is None or (lp, t, rp) not in A:
                        continue
                    At = A[(lp, t, rp)]
                    n = sel.size
                    # Z = As^T X At for every selected row
                    Z1 = (X[sel].reshape(n * ml, mlp) @ At).reshape(n, ml, -1)
                    mr, mrp = As.shape[1], At.shape[1]
                    Z = (As.T @ Z1.transpose(1, 0, 2).reshape(ml, n * mrp)).reshape(mr, n, mrp).transpose(1, 0, 2)
                    if flops is not None:
                        flops[0] += 2.0 * n * ml * mlp * mrp + 2.0 * n * mr * ml * mrp
                    dout = mpo.dq[x + 1][outch[sel[0]]]
                    assert _qdiff(bond_r.q(r), bond_r.q(rp)) == dout
                    arr = out.block(dout, r, rp)
                    slots = [out.classes[dout]["slot"][b] for b in outch[sel]]
                    _scatter_into(arr, slots, w[sel], Z)
    return out


def update_right(env: Env, A: dict, bond_l: Bond, mpo: MPO, x: int, flops=None):
    """R_x from R_{x+1} and the site tensor A of site x (dict (l, s, r) -> block)."""
    out = Env(bond_l, mpo.dq[x])
    groups = _groups(mpo.W[x], by_left=False)
    for d, (rows, C) in _mix_rows(env, groups, mpo.dq[x + 1]).items():
        ops = np.array([MPO.op_matrix(k[1]) for k in rows])
        outch = np.array([k[0] for k in rows])
        for (r, rp), data in env.classes[d]["blocks"].items():
            n_ch, mr, mrp = data.shape
            Y = (C @ data.reshape(n_ch, -1)).reshape(len(rows), mr, mrp)
            for s in range(4):
                l = bond_l.find(_sub(env.bond.q(r), SITE_QN[s]))
                if l is None or (l, s, r) not in A:
                    continue
                As = A[(l, s, r)]
                for t in range(4):
                    w = ops[:, s, t]
                    sel = np.nonzero(w)[0]
                    if sel.size == 0:
                        continue
                    lp = bond_l.find(_sub(env.bond.q(rp), SITE_QN[t]))
                    if lp is None or (lp, t, rp) not in A:
                        continue
                    At = A[(lp, t, rp)]
                    n = sel.size
                    ml, mlp = As.shape[0], At.shape[0]
                    # Z = As Y At^T for every selected row
                    Z1 = (Y[sel].reshape(n * mr, mrp) @ At.T).reshape(n, mr, mlp)
                    Z = (As @ Z1.transpose(1, 0, 2).reshape(mr, n * mlp)).reshape(ml, n, mlp).transpose(1, 0, 2)
                    if flops is not None:
                        flops[0] += 2.0 * n * mr * mrp * mlp + 2.0 * n * ml * mr * mlp
                    dout = mpo.dq[x][outch[sel[0]]]
                    assert _qdiff(bond_l.q(l), bond_l.q(lp)) == dout
                    arr = out.block(dout, l, lp)
                    slots = [out.classes[dout]["slot"][a] for a in outch[sel]]
                    _scatter_into(arr, slots, w[sel], Z)
    return out


# ------------------------------------------------------------------- the MPS --
def mps_blocks(mps):
    """(bonds, site block dicts) from {bonds: [[(N, 2Sz, dim)...]...], sites: [flat...]}."""
    bonds = [Bond(b) for b in mps["bonds"]]
    A = [unpack(bonds[k], bonds[k + 1], SITE_QN, mps["sites"][k]) for k in range(len(mps["sites"]))]
    return bonds, A


def environments(mpo: MPO, mps, k, progress=None):
    """(L_k, R_{k+2}) for the two-site step on sites (k, k+1)."""
    bonds, A = mps_blocks(mps)
    L = len(A)
    envL = left_boundary(mpo, bonds[0])
    for x in range(k):
        envL = update_left(envL, A[x], bonds[x + 1], mpo, x)
        if progress:
            progress(f"left environment cut {x + 1} of {k}")
    envR = right_boundary(mpo, bonds[L])
    for x in range(L - 1, k + 1, -1):
        envR = update_right(envR, A[x], bonds[x], mpo, x)
        if progress:
            progress(f"right environment cut {x} (down to {k + 2})")
    return envL, envR


# --------------------------------------------------------------------- sigma --
class TwoSite:
    """The two-site H_eff of step k: environments, the mixed left / right rows and psi layout."""

    def __init__(self, mpo: MPO, mps, k, progress=None):
        self.mpo, self.k = mpo, k
        bonds = [Bond(b) for b in mps["bonds"]]
        self.bl, self.br = bonds[k], bonds[k + 2]
        self.envL, self.envR = environments(mpo, mps, k, progress)
        gl = _groups(mpo.W[k], by_left=True)     # (beta, O) <- alpha
        gr = _groups(mpo.W[k + 1], by_left=False)  # (beta, O') <- gamma
        self.left_rows = {}   # beta -> list of (class d, opmatrix, sources)
        self.right_rows = {}
        for (beta, opk), srcs in gl.items():
            d = mpo.dq[k][srcs[0][0]]
            if d in self.envL.classes:
                self.left_rows.setdefault(beta, []).append((d, MPO.op_matrix(opk), srcs))
        for (beta, opk), srcs in gr.items():
            d = mpo.dq[k + 2][srcs[0][0]]
            if d in self.envR.classes:
                self.right_rows.setdefault(beta, []).append((d, MPO.op_matrix(opk), srcs))
        self.betas = [b for b in sorted(self.left_rows) if b in self.right_rows]
        self._cache = {}

    def _mixed(self, side, beta, i, bra):
        """Block (bra, bra - dq) of the i-th mixed row of beta on one side, or None."""
        key = (side, beta, i, bra)
        if key in self._cache:
            return self._cache[key]
        env = self.envL if side == 0 else self.envR
        d, _, srcs = (self.left_rows if side == 0 else self.right_rows)[beta][i]
        ket = env.bond.find(_sub(env.bond.q(bra), d))
        out = None
        if ket is not None:
            cl = env.classes[d]
            arr = cl["blocks"].get((bra, ket))
            if arr is not None:
                out = np.zeros(arr.shape[1:])
                for s, c in srcs:
                    out += c * arr[cl["slot"][s]]
        self._cache[key] = (ket, out)
        return ket, out

    def sigma_block(self, psi_blocks, a, s1, s2, b, flops=None):
        """Output block (a, 4 s1 + s2, b) of sigma = H_eff psi."""
        out = np.zeros((self.bl.dim(a), self.br.dim(b)))
        for beta in self.betas:
            lrows, rrows = self.left_rows[beta], self.right_rows[beta]
            for i, (dl, Ol, _) in enumerate(lrows):
                ap, X = self._mixed(0, beta, i, a)
                if X is None:
                    continue
                for t1 in range(4):
                    wl = Ol[s1, t1]
                    if wl == 0.0:
                        continue
                    for t2 in range(4):
                        # right rows of this beta acting s2 <- t2, summed per class
                        ysum = {}
                        for j, (dr, Or, _) in enumerate(rrows):
                            wr = Or[s2, t2]
                            if wr == 0.0:
                                continue
                            bp, Y = self._mixed(1, beta, j, b)
                            if Y is None:
                                continue
                            if bp in ysum:
                                ysum[bp] = ysum[bp] + wr * Y
                            else:
                                ysum[bp] = wr * Y
                        for bp, Ys in ysum.items():
                            blk = psi_blocks.get((ap, 4 * t1 + t2, bp))
                            if blk is None:
                                continue
                            T = X @ blk
                            out += wl * (T @ Ys.T)
                            if flops is not None:
                                flops[0] += 2.0 * X.shape[0] * X.shape[1] * blk.shape[1]
                                flops[0] += 2.0 * X.shape[0] * blk.shape[1] * Ys.shape[0]
        return out

    def output_blocks(self):
        return [(l, p, r) for l, p, r, *_ in slab_blocks(self.bl, self.br, twosite_qn())]

    def sigma(self, psi_flat, blocks=None, flops=None):
        """sigma as a slab-layout vector (blocks=None) or dict of the requested blocks."""
        pb = unpack(self.bl, self.br, twosite_qn(), psi_flat)
        want = self.output_blocks() if blocks is None else blocks
        res = {}
        for (a, p, b) in want:
            res[(a, p, b)] = self.sigma_block(pb, a, p // 4, p % 4, b, flops)
        if blocks is None:
            return pack(self.bl, self.br, twosite_qn(), res)
        return res

    def diag(self, blocks=None):
        """Diagonal of H_eff as a slab-layout vector (blocks=None) or dict of the requested blocks."""
        res = {}
        for (a, p, b) in (self.output_blocks() if blocks is None else blocks):
            s1, s2 = p // 4, p % 4
            D = np.zeros((self.bl.dim(a), self.br.dim(b)))
            for beta in self.betas:
                for i, (dl, Ol, _) in enumerate(self.left_rows[beta]):
                    if dl != (0, 0) or Ol[s1, s1] == 0.0:
                        continue
                    _, X = self._mixed(0, beta, i, a)
                    if X is None:
                        continue
                    for j, (dr, Or, _) in enumerate(self.right_rows[beta]):
                        if dr != (0, 0) or Or[s2, s2] == 0.0:
                            continue
                        _, Y = self._mixed(1, beta, j, b)
                        if Y is None:
                            continue
                        D += Ol[s1, s1] * Or[s2, s2] * np.outer(np.diag(X), np.diag(Y))
            res[(a, p, b)] = D
        if blocks is not None:
            return res
        return pack(self.bl, self.br, twosite_qn(), res)


def twosite_from_sites(mps, k):
    """psi[a s1 s2 b] = sum_m A_k[a s1 m] A_{k+1}[m s2 b] in slab layout."""
    bonds, A = mps_blocks(mps)
    bl, bm, br = bonds[k], bonds[k + 1], bonds[k + 2]
    out = {}
    for (a, s1, m), X in A[k].items():
        for s2 in range(4):
            b = br.find(_add(bm.q(m), SITE_QN[s2]))
            if b is None or (m, s2, b) not in A[k + 1]:
                continue
            key = (a, 4 * s1 + s2, b)
            prod = X @ A[k + 1][(m, s2, b)]
            out[key] = out[key] + prod if key in out else prod
    return pack(bl, br, twosite_qn(), out)


def right_orthonormality_error(mps, first):
    """max over sites x >= first and left sectors l of |sum_s A_s A_s^T - 1| (the
    right block states at every cut >= first are orthonormal when this is ~0)."""
    bonds, A = mps_blocks(mps)
    err = 0.0
    for x in range(first, len(A)):
        for l in range(len(bonds[x])):
            G = np.zeros((bonds[x].dim(l), bonds[x].dim(l)))
            for (ll, s, r), X in A[x].items():
                if ll == l:
                    G += X @ X.T
            err = max(err, float(np.max(np.abs(G - np.eye(G.shape[0])))))
    return err
