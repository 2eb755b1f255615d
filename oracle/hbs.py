"""HBS compression of G and its inverse by scattering matrices (oracle side).

TEST INFRASTRUCTURE.  Plain numpy/scipy transcription of the paper's method:

* Tree (Sec. 3.1, 3.2): uniform binary tree with 2^L leaves; the root is the
  whole grid; cuts alternate vertical (split x1) at even levels and horizontal
  (split x2) at odd levels; children of box t on level l are boxes 2t (the
  half with the smaller coordinates, alpha) and 2t+1 (beta) on level l+1.
* Compression (Sec. 3.2): only the b-independent matrix G of eq. (Gmat) is
  compressed: 4th order for the preconditioner; the direct-solver
  experiments (Sec. 6) compress higher orders, whose correction stencils
  reach up to 3 lattice steps, so every block (leaf, proxy, sibling) takes
  the corrected entries, and the proxy ring must be at least as wide as the
  stencil.  Leaf row ID of G(I_tau, proxy ring) (eqs.
  (leafid), (proxy)); parent row ID of G([J_alpha, J_beta], proxy ring)
  (eq. (parentid)); sibling blocks G_ab = G(J_alpha, J_beta) (eq. (sibint)).
  Translation invariance: one ID per level, done on box 0 in box-local
  lattice coordinates and shared by all boxes of the level.  V_tau = U_tau by
  the symmetry of G; since G is complex symmetric (not Hermitian) the row
  basis is used transposed: V* := U^T.
* ID (Sec. 2.1): CPQR of A^T (LAPACK zgeqp3 via scipy); the local tolerance
  is eps * ||A||_F (Remark on the local tolerance): the rank is the first k
  with |R_kk| <= eps ||A||_F.  tol = 0 selects the exact full-rank form
  (U = I, J = all candidates), in which the HBS matrix equals G.
* Build: Algorithm 1 (eqs. (localsol_leaf), (smat_leaf), (localsol), (smat)).
  Optionally (the remark after Algorithm 2's description, eq. (blockinv))
  the merge inverse X_tau by the Woodbury formula on a low-rank sibling
  block G_ab ~= L R^T (a row ID of G_ab at its own tolerance).  As printed,
  eq. (blockinv) leaves out the scattering matrices: with
  P = diag(S_a L_ab, S_b L_ba) and Q = [[0, R_ab^T], [R_ba^T, 0]] the
  merge matrix is I + P Q, so X_tau = I - P (I + Q P)^{-1} Q.
* Apply: Algorithm 2, loops read as: up l = L-1..1, top solve at the root,
  down l = 1..L-1, then the leaves.  Also its exact transpose and the HBS
  forward matvec of G^eps.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import quadrature as quad


class Tree:
    def __init__(self, n: int, leaf: int, levels: int | None = None):
        p = n // leaf
        if leaf * p != n or p & (p - 1):
            raise ValueError("n / leaf must be a power of two")
        self.n, self.leaf = n, leaf
        # default: square leaves of side `leaf`; `levels` may stop the
        # bisection earlier (then the leaves may be 2:1 rectangles)
        self.L = 2 * int(round(np.log2(p))) if levels is None else int(levels)
        if not 1 <= self.L <= 2 * int(round(np.log2(n))):
            raise ValueError("bad number of levels")

    def box(self, level: int, t: int):
        """(ox, oy, sx, sy) of box t on a level, in lattice units."""
        ox, oy, sx, sy = 0, 0, self.n, self.n
        for m in range(1, level + 1):
            bit = (t >> (level - m)) & 1
            if (m - 1) % 2 == 0:  # vertical cut: split x1
                sx //= 2
                ox += bit * sx
            else:  # horizontal cut: split x2
                sy //= 2
                oy += bit * sy
        return ox, oy, sx, sy

    def tree_points(self, level: int, t: int):
        """Global indices in tree order: children concatenated, leaves row-major."""
        if level == self.L:
            return self.points(level, t)
        return np.concatenate([self.tree_points(level + 1, 2 * t), self.tree_points(level + 1, 2 * t + 1)])

    def points(self, level: int, t: int):
        """Global grid indices of the box's nodes, box-local row-major order."""
        ox, oy, sx, sy = self.box(level, t)
        iy, ix = np.meshgrid(np.arange(sy), np.arange(sx), indexing="ij")
        return ((oy + iy) * self.n + (ox + ix)).reshape(-1)


def proxy_ring(sx: int, sy: int, w: int):
    """Lattice points of the w layers just outside an sx x sy box (box-local)."""
    pts = [(a, b) for b in range(-w, sy + w) for a in range(-w, sx + w)
           if not (0 <= a < sx and 0 <= b < sy)]
    return np.array(pts, dtype=np.int64)


def row_id(A, tol: float):
    """Row ID A ~= U A[J, :] with U[J, :] = I, by CPQR of A^T."""
    m = A.shape[0]
    if tol == 0:
        return np.arange(m), np.eye(m, dtype=complex)
    R, P = sla.qr(A.T, mode="r", pivoting=True)
    d = np.abs(np.diag(R))
    thr = tol * np.linalg.norm(A)
    small = np.nonzero(d <= thr)[0]
    k = int(small[0]) if small.size else d.size
    k = max(k, 1)
    J = P[:k]
    T = sla.solve_triangular(R[:k, :k], R[:k, k:])  # R11^{-1} R12
    U = np.zeros((m, k), dtype=complex)
    U[J, :] = np.eye(k)
    U[P[k:], :] = T.T
    return J, U


class Compression:
    """Per-level shared factors {J_l, U_l, G_ab,l} and the leaf block of G."""

    def __init__(self, n: int, kappa: float, leaf: int, tol: float, w: int,
                 levels: int | None = None, order: int = 4):
        self.tree = T = Tree(n, leaf, levels)
        self.n, self.kappa, self.tol, self.w, self.order = n, kappa, tol, w, order
        self.h = 1.0 / n
        self.tau = quad.correction_weights(order, kappa * self.h)
        reach = max(max(abs(a), abs(b)) for a, b in self.tau)
        if reach > w:
            raise ValueError(f"order-{order} stencil reaches {reach} > proxy width {w}")
        L = T.L
        self.cand = {}   # level -> candidate rows (box-local lattice coords)
        self.skel = {}   # level -> skeleton coords (box-local)
        self.U = {}      # level -> (m x k) interpolation matrix
        self.J = {}
        for lev in range(L, 0, -1):
            ox, oy, sx, sy = T.box(lev, 0)
            if lev == L:
                iy, ix = np.meshgrid(np.arange(sy), np.arange(sx), indexing="ij")
                cand = np.stack([ix.reshape(-1), iy.reshape(-1)], axis=1)
            else:
                parts = []
                for c in (0, 1):
                    cx, cy, _, _ = T.box(lev + 1, c)
                    parts.append(self.skel[lev + 1] + np.array([cx - ox, cy - oy]))
                cand = np.concatenate(parts)
            A = self.proxy_block(cand, proxy_ring(sx, sy, w))
            J, U = row_id(A, tol)
            self.cand[lev], self.J[lev], self.U[lev] = cand, J, U
            self.skel[lev] = cand[J]
        # sibling blocks: G_ab on parent level l couples child 0 and child 1
        self.Gab = {}
        for lev in range(0, L):
            a = self.skel[lev + 1] + np.array(T.box(lev + 1, 0)[:2])
            b = self.skel[lev + 1] + np.array(T.box(lev + 1, 1)[:2])
            self.Gab[lev] = self.gblock(a, b)
        lx, ly, sx, sy = T.box(L, 0)
        self.Gleaf = self.gblock(self.cand[L], self.cand[L])

    def gblock(self, rows, cols):
        """Order-p entries h^2 (G(h|d|) [d != 0] + tau_d), d = col - row (eq. (Gmat))."""
        rows = np.asarray(rows).reshape(-1, 2)
        cols = np.asarray(cols).reshape(-1, 2)
        dx = cols[None, :, 0] - rows[:, None, 0]
        dy = cols[None, :, 1] - rows[:, None, 1]
        d = np.hypot(dx, dy)
        G = np.zeros(d.shape, dtype=complex)
        nz = d > 0
        G[nz] = quad.green(self.kappa, self.h * d[nz])
        for (ox, oy), t in self.tau.items():
            G[(dx == ox) & (dy == oy)] += t
        return self.h * self.h * G

    def proxy_block(self, rows, ring):
        """Columns whose span must hold every row of the box's off-diagonal
        block: plain G on the ring (Green's representation of all sources
        beyond the stencil's reach) and, for orders above 4, the corrected
        entries against the ring points themselves, which are the actual
        near neighbours (the ring is at least as wide as the stencil)."""
        A = self.gblock(rows, ring)
        if self.order == 4:
            return A
        tau = self.tau
        self.tau = {(0, 0): tau[(0, 0)]}
        try:
            G = self.gblock(rows, ring)
        finally:
            self.tau = tau
        return np.hstack([G, A])

    def ranks(self):
        return {lev: self.U[lev].shape[1] for lev in self.U}

    def matvec(self, x):
        """y = G^eps x, the HBS matrix applied to x (grid order)."""
        T, L = self.tree, self.tree.L
        x = np.asarray(x, dtype=complex).reshape(-1)
        qt = {}
        for t in range(2 ** L):
            qt[(L, t)] = self.U[L].T @ x[T.points(L, t)]
        for lev in range(L - 1, 0, -1):
            for t in range(2 ** lev):
                qt[(lev, t)] = self.U[lev].T @ np.concatenate([qt[(lev + 1, 2 * t)], qt[(lev + 1, 2 * t + 1)]])
        wt = {}
        for lev in range(0, L):
            G = self.Gab[lev]
            for t in range(2 ** lev):
                qa, qb = qt[(lev + 1, 2 * t)], qt[(lev + 1, 2 * t + 1)]
                wa, wb = G @ qb, G.T @ qa
                if lev > 0:
                    inc = self.U[lev] @ wt[(lev, t)]
                    wa, wb = wa + inc[:qa.size], wb + inc[qa.size:]
                wt[(lev + 1, 2 * t)], wt[(lev + 1, 2 * t + 1)] = wa, wb
        y = np.zeros_like(x)
        for t in range(2 ** L):
            idx = T.points(L, t)
            y[idx] = self.Gleaf @ x[idx] + self.U[L] @ wt[(L, t)]
        return y


def woodbury_merge(Sa, Sb, L, Rt):
    """X_tau = [[I, S_a G_ab], [S_b G_ab^T, I]]^{-1} for G_ab = L Rt (eq.
    (blockinv) with the S factors): G_ba = G_ab^T = Rt^T L^T, so L_ab = L,
    R_ab^T = Rt, L_ba = Rt^T, R_ba^T = L^T."""
    ca, cb, r = Sa.shape[0], Sb.shape[0], L.shape[1]
    P = sla.block_diag(Sa @ L, Sb @ Rt.T)
    Q = np.block([[np.zeros((r, ca)), Rt], [L.T, np.zeros((r, cb))]])
    return np.eye(ca + cb) - P @ np.linalg.solve(np.eye(2 * r) + Q @ P, Q)


class Inverse:
    """Algorithm 1 (build) and Algorithm 2 (apply) for (I + B G^eps)^{-1}.

    lowrank_tol: None forms X_tau by inverting the merge matrix; a number
    uses woodbury_merge with G_ab ~= L Rt, the row ID of G_ab at that
    tolerance (L = U, Rt = G_ab[J, :])."""

    def __init__(self, comp: Compression, b, lowrank_tol=None):
        self.comp = comp
        self.lowrank = {}
        if lowrank_tol is not None:
            for lev, G in comp.Gab.items():
                J, Ug = row_id(G, lowrank_tol)
                self.lowrank[lev] = (Ug, G[J, :])
        T, L = comp.tree, comp.tree.L
        self.B = comp.kappa ** 2 * np.asarray(b, dtype=float).reshape(-1)
        self.X, self.S = {}, {}
        for t in range(2 ** L):
            Bt = self.B[T.points(L, t)]
            X = np.linalg.inv(np.eye(Bt.size) + Bt[:, None] * comp.Gleaf)
            self.X[(L, t)] = X
            self.S[(L, t)] = comp.U[L].T @ X @ (Bt[:, None] * comp.U[L])
        for lev in range(L - 1, -1, -1):
            Gab = comp.Gab[lev]
            for t in range(2 ** lev):
                Sa, Sb = self.S[(lev + 1, 2 * t)], self.S[(lev + 1, 2 * t + 1)]
                ca, cb = Sa.shape[0], Sb.shape[0]
                if lowrank_tol is None:
                    M = np.block([[np.eye(ca), Sa @ Gab], [Sb @ Gab.T, np.eye(cb)]])
                    X = np.linalg.inv(M)
                else:
                    X = woodbury_merge(Sa, Sb, *self.lowrank[lev])
                self.X[(lev, t)] = X
                if lev > 0:
                    D = sla.block_diag(Sa, Sb)
                    self.S[(lev, t)] = comp.U[lev].T @ X @ D @ comp.U[lev]

    def _Ghat(self, lev, v, ca):
        G = self.comp.Gab[lev]
        return np.concatenate([G @ v[ca:], G.T @ v[:ca]])

    def apply(self, f):
        """q = M f (Algorithm 2)."""
        comp, T, L = self.comp, self.comp.tree, self.comp.tree.L
        f = np.asarray(f, dtype=complex).reshape(-1)
        r, rt = {}, {}
        for t in range(2 ** L):
            r[t] = self.X[(L, t)] @ f[T.points(L, t)]
            rt[(L, t)] = comp.U[L].T @ r[t]
        for lev in range(L - 1, 0, -1):
            for t in range(2 ** lev):
                v = np.concatenate([rt[(lev + 1, 2 * t)], rt[(lev + 1, 2 * t + 1)]])
                rt[(lev, t)] = comp.U[lev].T @ (self.X[(lev, t)] @ v)
        wt = {}
        v = np.concatenate([rt[(1, 0)], rt[(1, 1)]])
        ca = rt[(1, 0)].size
        w = self._Ghat(0, self.X[(0, 0)] @ v, ca)
        wt[(1, 0)], wt[(1, 1)] = w[:ca], w[ca:]
        for lev in range(1, L):
            for t in range(2 ** lev):
                Sa, Sb = self.S[(lev + 1, 2 * t)], self.S[(lev + 1, 2 * t + 1)]
                ca = Sa.shape[0]
                v = np.concatenate([rt[(lev + 1, 2 * t)], rt[(lev + 1, 2 * t + 1)]])
                Uw = comp.U[lev] @ wt[(lev, t)]
                qt = self.X[(lev, t)] @ (v - np.concatenate([Sa @ Uw[:ca], Sb @ Uw[ca:]]))
                w = self._Ghat(lev, qt, ca) + Uw
                wt[(lev + 1, 2 * t)], wt[(lev + 1, 2 * t + 1)] = w[:ca], w[ca:]
        q = np.zeros_like(f)
        for t in range(2 ** L):
            idx = T.points(L, t)
            q[idx] = r[t] - self.X[(L, t)] @ (self.B[idx] * (comp.U[L] @ wt[(L, t)]))
        return q

    def apply_transpose(self, g):
        """q = M^T g: the steps of Algorithm 2 transposed in reverse order."""
        comp, T, L = self.comp, self.comp.tree, self.comp.tree.L
        g = np.asarray(g, dtype=complex).reshape(-1)
        UL = comp.U[L]
        wb = {}
        for t in range(2 ** L):
            idx = T.points(L, t)
            wb[(L, t)] = -UL.T @ (self.B[idx] * (self.X[(L, t)].T @ g[idx]))
        vb = {}
        for lev in range(L - 1, 0, -1):
            for t in range(2 ** lev):
                Sa, Sb = self.S[(lev + 1, 2 * t)], self.S[(lev + 1, 2 * t + 1)]
                ca = Sa.shape[0]
                wc = np.concatenate([wb[(lev + 1, 2 * t)], wb[(lev + 1, 2 * t + 1)]])
                qb = self._Ghat(lev, wc, ca)
                xq = self.X[(lev, t)].T @ qb
                wb[(lev, t)] = comp.U[lev].T @ wc - comp.U[lev].T @ np.concatenate(
                    [Sa.T @ xq[:ca], Sb.T @ xq[ca:]])
                vb[(lev, t)] = qb
        ca = comp.U[1].shape[1]
        wc = np.concatenate([wb[(1, 0)], wb[(1, 1)]])
        rtb = {}
        x = self.X[(0, 0)].T @ self._Ghat(0, wc, ca)
        rtb[(1, 0)], rtb[(1, 1)] = x[:ca], x[ca:]
        for lev in range(1, L):
            for t in range(2 ** lev):
                ca = comp.U[lev + 1].shape[1]
                x = self.X[(lev, t)].T @ (vb[(lev, t)] + comp.U[lev] @ rtb[(lev, t)])
                rtb[(lev + 1, 2 * t)], rtb[(lev + 1, 2 * t + 1)] = x[:ca], x[ca:]
        q = np.zeros_like(g)
        for t in range(2 ** L):
            idx = T.points(L, t)
            q[idx] = self.X[(L, t)].T @ (g[idx] + UL @ rtb[(L, t)])
        return q
