"""Plain CPU FP64 oracle of two-site (two-tensor) TDVP on the binary tree
tensor network, with SVD truncation of the bond between the two updated
tensors (arXiv 2210.03763, Sec. "Tensor network simulations": the tree
network is evolved by TDVP with a two-tensor update, the bond dimension chi
being the convergence knob).

TEST INFRASTRUCTURE.  Only tests/ may import this module; the device's
two-site update (ttn_config.update) is checked against it.  It reuses the single-site oracle's tree, environments and
Lanczos exponential (the same test-only package) and adds the two-site
effective Hamiltonian, the SVD split and the two-site sweep.

Method (the projector-splitting TDVP of Haegeman et al. 2016 in the tree form
of Bauernfeind and Aichhorn 2020, both cited by the paper):
  * the tangent-space projector of the two-site manifold of a tree is the sum
    of the two-site projectors of its edges minus deg(v) - 1 single-site
    projectors of every node v (the edges meeting at v overlap in v);
  * a half-step S(tau) walks the tree depth first from the root.  Every edge
    (v, parent u) gets one forward update of its merged tensor,
    Theta <- exp(-i tau H_eff2) Theta, and is split again by a truncated SVD;
    between two edge updates that meet at a node, that node's centre tensor
    is evolved backward, exp(+i tau H_eff1).  So inner nodes are evolved
    backward twice, the root once, bottom nodes never;
  * one step is S(dt/2) followed by its exact reverse S*(dt/2), with H frozen
    at the step midpoint, as for the single-site integrator.
Readings (the paper gives no truncation rule): a split keeps the
min(chi, rank limit) largest singular values, exact zeros included, so that
the padded link dimensions of the tree stay fixed (the upper nodes carry no
physical legs, so a bond can only grow inside dimensions its neighbours
already have); with cutoff > 0 values below cutoff * s_max are dropped as
well.  The kept values are rescaled to the norm of the untruncated tensor,
and the discarded weight (sum of the dropped s^2 over sum s^2) is recorded
per split.

Pins: tests/test_oracle_two_site.py (the dense state-vector evolution at
maximal chi from an undressed product state, the best rank-k approximation
of a split against an eigendecomposition of Theta Theta^dag, energy
conservation for a constant H, norm and discarded-weight bookkeeping at
truncated chi).  Beyond those, the truncated evolution has no closed form:
parity unpinned there.
"""
from __future__ import annotations

from typing import List

import torch

from .ttn_oracle import CDT, OracleTTN, on_P, on_leg, qr_toward


def _op4(axis, M, X):
    """M applied on one leg of a four-leg tensor X[l, r, s, p]."""
    if axis == 0:
        return torch.einsum("ab,brsp->arsp", M, X)
    if axis == 1:
        return torch.einsum("ab,lbsp->lasp", M, X)
    if axis == 2:
        return torch.einsum("ab,lrbp->lrap", M, X)
    return torch.einsum("ab,lrsb->lrsa", M, X)


def truncated_split(Theta, chi: int, cutoff: float = 0.0):
    """Theta[l, r, s, p] = sum_k A[l, r, k] C[k, s, p] truncated to at most
    chi terms (and to values >= cutoff * s_max).  Returns (U, S, Vh, kept,
    discarded weight), U[(l r), k] and Vh[k, (s p)] with orthonormal columns
    and rows, S the kept singular values rescaled to the norm of Theta."""
    DL, DR, DS, DP = Theta.shape
    M = Theta.reshape(DL * DR, DS * DP)
    U, s, Vh = torch.linalg.svd(M, full_matrices=False)
    k = min(chi, s.shape[0])
    if cutoff > 0.0 and float(s[0]) > 0.0:
        k = max(1, min(k, int((s >= cutoff * s[0]).sum())))
    total = float((s ** 2).sum())
    kept = float((s[:k] ** 2).sum())
    disc = float((s[k:] ** 2).sum()) / total if total > 0.0 else 0.0
    S = s[:k] * (total / kept) ** 0.5 if kept > 0.0 else s[:k]
    return U[:, :k], S, Vh[:k, :], k, disc


class TwoSiteTTN(OracleTTN):
    """The single-site oracle's network and environments with the two-site
    sweep; build it like OracleTTN (init_product with eps = 0 gives the
    undressed product state)."""

    def __init__(self, *args, cutoff: float = 0.0, **kw):
        super().__init__(*args, **kw)
        self.cutoff = cutoff
        self.discarded: List[float] = []

    # -- the merged tensor of edge (v, parent u) -----------------------------
    def merge(self, v):
        tr = self.tree
        u, leg = tr.parent[v], tr.leg_in_parent(v)
        if leg == 0:
            return torch.einsum("lrk,ksp->lrsp", self.T[v], self.T[u])
        return torch.einsum("lrk,skp->lrsp", self.T[v], self.T[u])

    def heff2(self, v):
        """Theta -> H_eff2 Theta for edge (v, parent u), Theta[l, r, s, p]
        with l, r the legs of v's children, s the leg of v's sibling and p
        the parent leg of u: block terms of the four outer links, every pair
        V_ij n_i n_j with i and j below different outer links of v and u,
        and n_i (x) W_i on p for every site below u."""
        tr = self.tree
        u, leg = tr.parent[v], tr.leg_in_parent(v)
        HL, NL = self.child_env(v, 0)
        HR, NR = self.child_env(v, 1)
        HS, NS = self.child_env(u, 1 - leg)
        HP, WP = self.parent_env(u)
        AR = {i: self.A_op(i, NR) for i in NL}
        ASl = {i: self.A_op(i, NS) for i in NL}
        ASr = {j: self.A_op(j, NS) for j in NR}

        def apply(X):
            out = _op4(0, HL, X) + _op4(1, HR, X) + _op4(2, HS, X) + _op4(3, HP, X)
            for i, Ni in NL.items():
                Y = _op4(0, Ni, X)
                out = out + _op4(1, AR[i], Y) + _op4(2, ASl[i], Y) + _op4(3, WP[i], Y)
            for j, Nj in NR.items():
                Y = _op4(1, Nj, X)
                out = out + _op4(2, ASr[j], Y) + _op4(3, WP[j], Y)
            for k, Nk in NS.items():
                out = out + _op4(3, WP[k], _op4(2, Nk, X))
            return out
        return apply

    def update_edge(self, v, tau, centre_up: bool):
        """Forward two-site update of edge (v, u), then the split with the
        centre left in u (centre_up) or in v; rebuilds the environment of the
        link on the isometry's side."""
        tr = self.tree
        u, leg = tr.parent[v], tr.leg_in_parent(v)
        Theta = self.merge(v)
        Theta, info = self._expm(self.heff2(v), Theta, tau)
        self.stats.append(("edge", v, info["m"]))
        DL, DR, DS, DP = Theta.shape
        U, S, Vh, k, disc = truncated_split(Theta, self.tree.chi, self.cutoff)
        self.discarded.append(disc)
        Sc = S.to(CDT)
        if centre_up:
            A = U.reshape(DL, DR, k)
            C = (Sc.unsqueeze(1) * Vh).reshape(k, DS, DP)
        else:
            A = (U * Sc.unsqueeze(0)).reshape(DL, DR, k)
            C = Vh.reshape(k, DS, DP)
        self.T[v] = A
        self.T[u] = C if leg == 0 else C.permute(1, 0, 2).contiguous()
        if centre_up:
            self.build_up(v)
        else:
            self.build_down(v)

    # -- sweeps ------------------------------------------------------------
    def _visit2_fwd(self, v, tau):
        """Centre at the parent u of v on entry and on exit; every edge in
        the subtree of v and the edge (v, u) updated once."""
        tr = self.tree
        u, leg = tr.parent[v], tr.leg_in_parent(v)
        if not tr.is_bottom(v):
            Q, R = qr_toward(self.T[u], leg)     # centre down to v
            self.T[u] = Q
            self.T[v] = on_P(R, self.T[v])
            self.build_down(v)
            c0, c1 = tr.children[v]
            self._visit2_fwd(c0, tau)
            self.evolve_node(v, -tau)
            self._visit2_fwd(c1, tau)
            self.evolve_node(v, -tau)
        self.update_edge(v, tau, centre_up=True)

    def _visit2_bwd(self, v, tau):
        """The exact reverse of _visit2_fwd."""
        tr = self.tree
        u, leg = tr.parent[v], tr.leg_in_parent(v)
        if tr.is_bottom(v):
            self.update_edge(v, tau, centre_up=True)
            return
        self.update_edge(v, tau, centre_up=False)
        c0, c1 = tr.children[v]
        self.evolve_node(v, -tau)
        self._visit2_bwd(c1, tau)
        self.evolve_node(v, -tau)
        self._visit2_bwd(c0, tau)
        Q, R = qr_toward(self.T[v], 2)           # centre back up to u
        self.T[v] = Q
        self.build_up(v)
        self.T[u] = on_leg(leg, R, self.T[u])

    def sweep_fwd(self, tau):
        tr = self.tree
        c0, c1 = tr.children[tr.root]
        self._visit2_fwd(c0, tau)
        self.evolve_node(tr.root, -tau)
        self._visit2_fwd(c1, tau)

    def sweep_bwd(self, tau):
        tr = self.tree
        c0, c1 = tr.children[tr.root]
        self._visit2_bwd(c1, tau)
        self.evolve_node(tr.root, -tau)
        self._visit2_bwd(c0, tau)


def build(w, cutoff: float = 0.0) -> TwoSiteTTN:
    """Two-site oracle state from a workload description (its dressing is
    applied as given; eps = 0 leaves the undressed product state)."""
    st = TwoSiteTTN(w.n_sites, w.d, w.chi, w.pos_xy, w.leaf_order, w.c6, w.r_cut, w.leak_ratio,
                    w.krylov_dim, getattr(w, "gamma", 0.0), cutoff=cutoff)
    st.init_product(w.init_product, w.dress_eps, w.dress_noise)
    return st
