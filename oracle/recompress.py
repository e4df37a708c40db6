"""Algebraic recompression of the interpolation H^2 matrix.  FP64, NumPy.
TEST INFRASTRUCTURE ONLY.

The paper leaves more advanced approximations for later (the GCA-H^2 variant
in the section on distributed matrix setup, the recompression algorithm in the
outlook, whose weight matrices follow the patterns of the forward
transformation and of the interaction phase).  The method itself is not given
in the paper, so this module follows the standard construction for nested
bases and states every step:

1. Orthogonalisation (bottom up, the pattern of the forward transformation):
   a leaf basis is factored V_tau = Q_tau R_tau (QR); a parent's stacked
   matrix [R_c1 E_c1; R_c2 E_c2] is factored Q R_tau and the blocks of Q are
   the new, orthonormal transfer matrices.  Then V-bar_tau = Q-bar_tau R_tau for
   every cluster, and S_{tau sigma} becomes R_tau S R_sigma^T: the represented
   matrix does not change.
2. Weights (top down): the Gram matrix of everything the row cluster tau
   carries in the orthonormal basis, G_tau = E'_tau G_parent E'_tau^T +
   sum over admissible (tau, sigma) of (R_tau S R_sigma^T)(R_tau S R_sigma^T)^T
   (the pattern of the interaction phase).
3. Truncation (bottom up): a leaf keeps the dominant eigenvectors U of G_tau;
   a parent first expresses its basis in the children's truncated bases,
   P_tau = [T_c1 E'_c1; T_c2 E'_c2] with T_c the coefficients of Q-bar_c in the
   new basis of c, then keeps the dominant eigenvectors of P G P^T; their
   blocks are the new transfer matrices and T_tau = U^T P_tau.
4. Coupling: S'_{tau sigma} = (T_tau R_tau) S (T_sigma R_sigma)^T.

Rank rule, per cluster: eps = 0 keeps every direction (pure orthogonalisation:
T = I, the orthonormal bases of step 1, rank min(|tau|, k) at a leaf and
min(rank c1 + rank c2, k) at a parent, unless max_rank cuts them); eps > 0
keeps the eigenvalues lambda_i > eps^2 lambda_max of that cluster's matrix;
max_rank > 0 caps the rank.  The discarded eigenvalues sum to `discarded`;
the Frobenius error of the admissible part then satisfies
||G~ - G~'||_F^2 <= 2 * discarded (row and column projections, G~ symmetric).
Real kernels only (test space = trial space, so one set of bases serves rows
and columns).
"""
from __future__ import annotations

import numpy as np


def _eig_desc(A):
    lam, U = np.linalg.eigh(0.5 * (A + A.T))
    order = np.argsort(lam)[::-1]
    return lam[order], U[:, order]


def _rank(lam, eps, cap, full):
    if eps == 0.0:
        r = full
    elif lam.size == 0 or lam[0] <= 0.0:
        r = 0
    else:
        r = int(np.count_nonzero(lam > eps * eps * lam[0]))
    if cap > 0:
        r = min(r, cap)
    return r


class Recompressed:
    """Nested orthonormal bases of variable rank: leaf bases Vn[c] (|c| x r_c),
    transfers En[c] (r_c x r_parent), couplings Sn[(t, s)] (r_t x r_s)."""

    def __init__(self, H, eps: float = 0.0, max_rank: int = 0):
        self.H = H
        k = H.k
        cl = H.tree.clusters
        by_level = sorted(cl, key=lambda c: c.level)
        up = by_level[::-1]                              # children before parents
        # 1. orthogonalisation
        Q, R, Eo = {}, {}, {}
        for c in up:
            if c.is_leaf:
                Q[c.id], R[c.id] = np.linalg.qr(H.V(c), mode="reduced")
            else:
                M = np.concatenate([R[ch.id] @ H.E(ch) for ch in c.children], 0)
                Qc, R[c.id] = np.linalg.qr(M, mode="reduced")
                row = 0
                for ch in c.children:
                    kc = R[ch.id].shape[0]
                    Eo[ch.id] = Qc[row:row + kc]
                    row += kc
        # 2. weights
        Gadm = {c.id: np.zeros((R[c.id].shape[0],) * 2) for c in cl}
        for t, s in H.adm:
            X = R[t.id] @ H.S(t, s) @ R[s.id].T
            Gadm[t.id] += X @ X.T
        G = {}
        for c in by_level:
            G[c.id] = Gadm[c.id] if c.parent is None else Eo[c.id] @ G[c.parent.id] @ Eo[c.id].T + Gadm[c.id]
        # 3. truncation
        T, self.Vn, self.En, self.rank = {}, {}, {}, {}
        self.discarded = 0.0
        for c in up:
            kc = R[c.id].shape[0]
            if eps == 0.0 and (max_rank <= 0 or max_rank >= kc):
                # nothing is cut: the orthogonalised bases themselves (T = I)
                T[c.id] = np.eye(kc)
                if c.is_leaf:
                    self.Vn[c.id] = Q[c.id]
                else:
                    for ch in c.children:
                        self.En[ch.id] = Eo[ch.id]
                self.rank[c.id] = kc
                continue
            if c.is_leaf:
                lam, U = _eig_desc(G[c.id])
                r = _rank(lam, eps, max_rank, kc)
                T[c.id] = U[:, :r].T
                self.Vn[c.id] = Q[c.id] @ U[:, :r]
            else:
                P = np.concatenate([T[ch.id] @ Eo[ch.id] for ch in c.children], 0)
                lam, U = _eig_desc(P @ G[c.id] @ P.T)
                r = _rank(lam, eps, max_rank, min(P.shape[0], kc))
                row = 0
                for ch in c.children:
                    rc = T[ch.id].shape[0]
                    self.En[ch.id] = U[row:row + rc, :r]
                    row += rc
                T[c.id] = U[:, :r].T @ P
            self.discarded += float(np.clip(lam[r:], 0.0, None).sum())
            self.rank[c.id] = r
        # 4. coupling
        Pf = {c.id: T[c.id] @ R[c.id] for c in cl}
        self.Sn = {(t.id, s.id): Pf[t.id] @ H.S(t, s) @ Pf[s.id].T for t, s in H.adm}
        self.max_rank = max(self.rank.values()) if self.rank else 0

    # ------------------------------------------------------------ forms
    def Vbar(self, c):
        if c.is_leaf:
            return self.Vn[c.id]
        return np.concatenate([self.Vbar(ch) @ self.En[ch.id] for ch in c.children], 0)

    def dense(self):
        H = self.H
        n = H.mesh.n
        G = np.zeros((n, n))
        for t, s in H.adm:
            G[np.ix_(t.idx, s.idx)] = self.Vbar(t) @ self.Sn[(t.id, s.id)] @ self.Vbar(s).T
        for t, s in H.inadm:
            G[np.ix_(t.idx, s.idx)] = H.N(t, s)
        return G

    def matvec(self, x):
        """y = G~' x by the three phases (forward, interaction, backward) on the
        recompressed bases."""
        H = self.H
        x = np.asarray(x, dtype=np.float64)
        y = np.zeros(H.mesh.n)
        xh, yh = {}, {}
        cl = sorted(H.tree.clusters, key=lambda c: c.level)
        for c in cl[::-1]:
            if c.is_leaf:
                xh[c.id] = self.Vn[c.id].T @ x[c.idx]
            else:
                xh[c.id] = sum(self.En[ch.id].T @ xh[ch.id] for ch in c.children)
            yh[c.id] = np.zeros(self.rank[c.id])
        for t, s in H.adm:
            yh[t.id] = yh[t.id] + self.Sn[(t.id, s.id)] @ xh[s.id]
        for t, s in H.inadm:
            y[t.idx] += H.N(t, s) @ x[s.idx]
        for c in cl:
            if c.parent is not None:
                yh[c.id] = yh[c.id] + self.En[c.id] @ yh[c.parent.id]
            if c.is_leaf:
                y[c.idx] += self.Vn[c.id] @ yh[c.id]
        return y
