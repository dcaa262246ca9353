"""Plain CPU FP64 oracle of single-site TDVP on a binary tree tensor network
under the time-dependent Rydberg Hamiltonian (arXiv 2210.03763).

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import or call this module.  It shares no
code with the device library: it receives the seeded input arrays and does
every step of the method itself, term by term, in complex128 torch CPU ops
(no blocking, fusion or reordering beyond regrouping a double sum), so that a
reader can check it against the paper by eye.

What it computes (paper sections in brackets):
  * Hamiltonian [Sec. "Modeling 88Sr quantum computers", Eq. (eq:ham) and
    Eq. (eq:c6)]: per site h_i(t) = Omega_i/2 (|1><r| + |r><1|) - Delta_i |r><r|
    (+ leak_ratio * Omega_i/2 (|leak><r| + |r><leak|) for d = 4)
    + Omega^x_i sigma^x + Omega^z_i sigma^z on the qubit levels, plus
    sum_{i<j} V_ij n_i n_j with V_ij = C6 / |r_i - r_j|^6 (sign and the
    double count of the printed double sum read as a single positive sum
    over pairs), optional cutoff radius.
  * Tree tensor network [Sec. "Tensor network simulations"]: binary tree,
    leaves along a Hilbert curve, N - 1 rank-3 nodes, bottom nodes own two
    physical legs, link dimension min(chi, d^s, d^(N-s)).
  * Tensor product operator [same section]: the Hamiltonian as a sum of
    one- and two-body terms, held per link as environment operators (a block
    Hamiltonian plus one n_i operator per site below the link, and from
    above a block Hamiltonian plus W_i = sum_{j above} V_ij n_j).
  * Time evolution [same section; the paper cites the projector-splitting
    TDVP of Haegeman et al. 2016 and its tree version by Bauernfeind and
    Aichhorn 2020]: single-site TDVP, one step = S(dt/2) followed by its
    exact reverse S*(dt/2) with H frozen at the step midpoint; local
    exponentials by Lanczos with full re-orthogonalisation; the small
    tridiagonal exponential through its symmetric eigendecomposition.
  * Observables: GHZ fidelity F = |<GHZ|psi>|^2 [Sec. on GHZ results],
    norm [open-system section], state overlap for C(p1, p2) [Tab. conv8x8],
    the total Rydberg population sum_i <n_i> [definitions of P_R and T_R].
  * Open system [Eq. (eq:hoqs)]: with a decay rate gamma > 0 every site's
    local term gains -i gamma |r><r|; the state is then not normalised
    (its norm is the no-decay probability), and the local exponentials use
    Arnoldi with a dense Hessenberg exponential instead of Lanczos.
  * Gradient of F with respect to the pulse table (the paper optimises
    pulses but gives no gradient method): the exact derivative of this
    discrete map, by reverse-mode automatic differentiation through every
    operation above (fidelity_gradient).

Parity pinned by tests/test_oracle_pins.py (dense state-vector evolution at
maximal chi, conservation laws, closed forms, padding invariance, blockade
limit, GHZ as a chi = 2 network); the gradient by tests/test_oracle_grad.py
(the dense Frechet-derivative gradient at maximal chi, central differences
of the map at truncated chi, exact zeros for dark atoms).  At truncated chi
the TDVP result has no closed form: only the invariants pin it ("parity
unpinned" beyond those).
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Tuple

import torch

CDT = torch.complex128
RDT = torch.float64

LANCZOS_BREAKDOWN = 1e-12   # relative: beta_{j+1} <= tol * (|alpha_j| + beta_j)
COMPLETION_TOL = 1e-8       # Gram-Schmidt acceptance for isometry completion


# ---------------------------------------------------------------------------
# Hamiltonian pieces
# ---------------------------------------------------------------------------

def local_ops(d: int):
    """X = |1><r| + h.c., n = |r><r|, Lk = |leak><r| + h.c. on {0, 1, r, leak}."""
    X = torch.zeros(d, d, dtype=CDT)
    n = torch.zeros(d, d, dtype=CDT)
    Lk = torch.zeros(d, d, dtype=CDT)
    X[1, 2] = X[2, 1] = 1.0
    n[2, 2] = 1.0
    if d >= 4:
        Lk[3, 2] = Lk[2, 3] = 1.0
    return X, n, Lk


def qubit_ops(d: int):
    """sigma^x = |0><1| + |1><0| and sigma^z = |0><0| - |1><1| on the qubit
    levels (Eq. (eq:ham)); zero on |r> and |leak>."""
    sx = torch.zeros(d, d, dtype=CDT)
    sz = torch.zeros(d, d, dtype=CDT)
    sx[0, 1] = sx[1, 0] = 1.0
    sz[0, 0] = 1.0
    sz[1, 1] = -1.0
    return sx, sz


def vdw_matrix(pos: torch.Tensor, c6: float, r_cut: float) -> torch.Tensor:
    """V_ij = C6 / d_ij^6 for i != j (d_ij Euclidean), 0 on the diagonal and
    beyond the cutoff radius when r_cut > 0."""
    N = pos.shape[0]
    V = torch.zeros(N, N, dtype=RDT)
    for i in range(N):
        for j in range(N):
            if i == j:
                continue
            dx = float(pos[i, 0] - pos[j, 0])
            dy = float(pos[i, 1] - pos[j, 1])
            dist = math.sqrt(dx * dx + dy * dy)
            if r_cut > 0 and dist > r_cut:
                continue
            V[i, j] = c6 / dist ** 6
    return V


def pulse_at(seg_edges, omega, delta, t: float):
    """Piecewise-constant drive: segment s with edges[s] <= t < edges[s+1];
    zero drive outside all segments."""
    S = len(seg_edges) - 1
    for s in range(S):
        if seg_edges[s] <= t < seg_edges[s + 1]:
            return omega[:, s], delta[:, s], s
    return torch.zeros(omega.shape[0], dtype=omega.dtype), torch.zeros(omega.shape[0], dtype=omega.dtype), -1


# ---------------------------------------------------------------------------
# elementary leg operations on a node tensor T[l, r, p]
# ---------------------------------------------------------------------------

def on_L(M, T):
    return torch.einsum("ab,brp->arp", M, T)


def on_R(M, T):
    return torch.einsum("ab,lbp->lap", M, T)


def on_P(M, T):
    return torch.einsum("ab,lrb->lra", M, T)


def on_leg(leg, M, T):
    return (on_L, on_R, on_P)[leg](M, T)


def proj(leg, Q, X):
    """<Q|X> over every leg but `leg`: E[a, b] = sum conj(Q[.., a, ..]) X[.., b, ..]."""
    if leg == 0:
        return torch.einsum("lrp,mrp->lm", Q.conj(), X)
    if leg == 1:
        return torch.einsum("lrp,lmp->rm", Q.conj(), X)
    return torch.einsum("lrp,lrq->pq", Q.conj(), X)


def qr_toward(T, leg):
    """Thin QR of T matricised with `leg` as the column index, with real
    positive diagonal of R:  T[.., a, ..] = sum_k Q[.., k, ..] R[k, a]."""
    perm = [i for i in range(3) if i != leg] + [leg]
    Tp = T.permute(*perm)
    shp = Tp.shape
    M = Tp.reshape(-1, shp[-1])
    Qm, R = torch.linalg.qr(M, mode="reduced")
    dg = torch.diagonal(R)
    mag = dg.abs()
    ph = torch.where(mag > 0, dg / torch.where(mag > 0, mag, torch.ones_like(mag)),
                     torch.ones_like(dg))
    Qm = Qm * ph.unsqueeze(0)
    R = ph.conj().unsqueeze(1) * R
    inv = [0, 0, 0]
    for k, p in enumerate(perm):
        inv[p] = k
    Q = Qm.reshape(shp).permute(*inv)
    return Q, R


# ---------------------------------------------------------------------------
# Lanczos exponential
# ---------------------------------------------------------------------------

def lanczos_expm(apply, v0, tau: float, m: int):
    """exp(-i tau H) v0 in the Krylov space of dimension <= m (H Hermitian).

    Three-term recurrence, then two full classical Gram-Schmidt passes
    against all previous basis vectors; happy breakdown when
    beta_{j+1} <= tol (|alpha_j| + beta_j).  The exponential of the real
    symmetric tridiagonal matrix T_m comes from its eigendecomposition."""
    beta0 = torch.linalg.vector_norm(v0)
    if float(beta0.detach()) == 0.0:
        return v0.clone(), dict(m=0, beta=[])
    V = [v0 / beta0]
    alphas: List[torch.Tensor] = []
    betas: List[torch.Tensor] = []
    for j in range(m):
        w = apply(V[j])
        a = torch.vdot(V[j].reshape(-1), w.reshape(-1)).real
        w = w - a * V[j]
        if j > 0:
            w = w - betas[j - 1] * V[j - 1]
        alphas.append(a)
        if j == m - 1:
            break
        for _ in range(2):
            coef = [torch.vdot(Vk.reshape(-1), w.reshape(-1)) for Vk in V]
            for ck, Vk in zip(coef, V):
                w = w - ck * Vk
        b = torch.linalg.vector_norm(w)
        bprev = betas[j - 1] if j > 0 else torch.zeros((), dtype=RDT)
        if float(b.detach()) <= LANCZOS_BREAKDOWN * (abs(float(a.detach())) + float(bprev.detach())):
            break
        betas.append(b)
        V.append(w / b)
    k = len(alphas)
    Tm = torch.diag(torch.stack(alphas))
    if k > 1:
        b = torch.stack(betas[:k - 1])
        Tm = Tm + torch.diag(b, 1) + torch.diag(b, -1)
    # exp(-i tau T) e_1 = U exp(-i tau Lambda) U^T e_1 for real symmetric T
    lam, U = torch.linalg.eigh(Tm)
    y = (U.to(CDT) * torch.exp(-1j * tau * lam)) @ U[0].to(CDT)
    out = torch.zeros_like(v0)
    for i in range(k):
        out = out + (beta0 * y[i]) * V[i]
    return out, dict(m=k, beta=[float(b.detach()) for b in betas])


def arnoldi_expm(apply, v0, tau: float, m: int):
    """exp(-i tau H) v0 in the Krylov space of dimension <= m for a general
    (non-Hermitian) H, as needed by the open-system Hamiltonian.

    Arnoldi: each new vector H v_j is orthogonalised against all previous
    basis vectors by two classical Gram-Schmidt passes, and the projection
    coefficients of both passes make up column j of the upper Hessenberg
    matrix H_m (the last column takes the first pass only, since no further
    basis vector is formed); h_{j+1,j} = ||w||, happy breakdown when
    h_{j+1,j} <= tol (|Re h_jj| + h_{j,j-1}) with the first-pass h_jj.  The
    small exponential exp(-i tau H_m) e_1 comes from the dense matrix
    exponential."""
    beta0 = torch.linalg.vector_norm(v0)
    if float(beta0.detach()) == 0.0:
        return v0.clone(), dict(m=0, beta=[])
    V = [v0 / beta0]
    Hm = torch.zeros(m + 1, m, dtype=CDT)
    k = 0
    for j in range(m):
        w = apply(V[j])
        coef = [torch.vdot(Vk.reshape(-1), w.reshape(-1)) for Vk in V]
        first_diag = coef[j]
        for i, ck in enumerate(coef):
            Hm[i, j] = Hm[i, j] + ck
        k = j + 1
        if j == m - 1:
            break
        for ck, Vk in zip(coef, V):
            w = w - ck * Vk
        coef = [torch.vdot(Vk.reshape(-1), w.reshape(-1)) for Vk in V]
        for i, (ck, Vk) in enumerate(zip(coef, V)):
            w = w - ck * Vk
            Hm[i, j] = Hm[i, j] + ck
        b = torch.linalg.vector_norm(w)
        bprev = float(Hm[j, j - 1].real) if j > 0 else 0.0
        if float(b) <= LANCZOS_BREAKDOWN * (abs(float(first_diag.real)) + bprev):
            break
        Hm[j + 1, j] = b
        V.append(w / b)
    y = torch.linalg.matrix_exp(-1j * tau * Hm[:k, :k])[:, 0]
    out = torch.zeros_like(v0)
    for i in range(k):
        out = out + (beta0 * y[i]) * V[i]
    return out, dict(m=k, beta=[float(Hm[i + 1, i].real) for i in range(k - 1)])


# ---------------------------------------------------------------------------
# tree
# ---------------------------------------------------------------------------

class Tree:
    """Binary tree over N = 2^K leaves.  Node (lvl, j) has id off[lvl] + j;
    level 0 nodes hold leaves 2j, 2j+1; node (lvl, j) with lvl >= 1 has
    children (lvl-1, 2j), (lvl-1, 2j+1); the root is the single top node."""

    def __init__(self, n_sites: int, d: int, chi: int, leaf_order):
        K = int(round(math.log2(n_sites)))
        if 1 << K != n_sites or n_sites < 2:
            raise ValueError("number of sites must be a power of two >= 2")
        self.N, self.d, self.chi, self.K = n_sites, d, chi, K
        self.leaf_site = [int(s) for s in leaf_order]
        if sorted(self.leaf_site) != list(range(n_sites)):
            raise ValueError("leaf order must be a permutation of the sites")
        self.off = []
        o = 0
        for lvl in range(K):
            self.off.append(o)
            o += n_sites >> (lvl + 1)
        self.n_nodes = o
        self.root = o - 1
        self.level, self.idx, self.parent, self.children = [], [], [], []
        for lvl in range(K):
            for j in range(n_sites >> (lvl + 1)):
                self.level.append(lvl)
                self.idx.append(j)
                self.parent.append(self.off[lvl + 1] + j // 2 if lvl + 1 < K else -1)
                self.children.append(None if lvl == 0 else
                                     (self.off[lvl - 1] + 2 * j, self.off[lvl - 1] + 2 * j + 1))
        self.dims = []
        for v in range(self.n_nodes):
            lvl = self.level[v]
            dc = d if lvl == 0 else self.link_dim(1 << lvl)
            self.dims.append((dc, dc, self.link_dim(1 << (lvl + 1))))
        for v in range(self.n_nodes):
            DL, DR, DP = self.dims[v]
            if DP > DL * DR:
                raise ValueError("inconsistent link dimensions")

    def link_dim(self, s: int) -> int:
        if s >= self.N:
            return 1
        return min(self.chi, self.d ** s, self.d ** (self.N - s))

    def is_bottom(self, v):
        return self.level[v] == 0

    def sites_below(self, v) -> List[int]:
        lvl, j = self.level[v], self.idx[v]
        w = 1 << (lvl + 1)
        return self.leaf_site[j * w:(j + 1) * w]

    def child_sites(self, v, side) -> List[int]:
        if self.is_bottom(v):
            return [self.leaf_site[2 * self.idx[v] + side]]
        return self.sites_below(self.children[v][side])

    def leg_in_parent(self, v) -> int:
        return self.idx[v] & 1

    def postorder(self) -> List[int]:
        out = []

        def rec(v):
            if not self.is_bottom(v):
                for c in self.children[v]:
                    rec(c)
            out.append(v)
        rec(self.root)
        return out

    def leaf_of_site(self, site) -> Tuple[int, int]:
        k = self.leaf_site.index(site)
        return k // 2, k & 1


# ---------------------------------------------------------------------------
# the TTN state with its environments
# ---------------------------------------------------------------------------

class OracleTTN:
    def __init__(self, n_sites, d, chi, pos_xy, leaf_order, c6=1.0, r_cut=0.0, leak_ratio=0.0,
                 krylov_dim=12, gamma=0.0):
        self.tree = Tree(n_sites, d, chi, leaf_order)
        self.d = d
        self.m = krylov_dim
        self.gamma = float(gamma)
        self.V = vdw_matrix(torch.as_tensor(pos_xy, dtype=RDT), c6, r_cut)
        self.X, self.n, self.Lk = local_ops(d)
        self.sx, self.sz = qubit_ops(d)
        self.leak_ratio = leak_ratio
        self.T: List[torch.Tensor] = [None] * self.tree.n_nodes
        self.up: Dict[int, dict] = {}
        self.down: Dict[int, dict] = {}
        self.omega_t = torch.zeros(n_sites, dtype=RDT)
        self.delta_t = torch.zeros(n_sites, dtype=RDT)
        self.omx_t = torch.zeros(n_sites, dtype=RDT)
        self.omz_t = torch.zeros(n_sites, dtype=RDT)
        self.stats = []
        self.qr_min = math.inf

    # -- initial state --------------------------------------------------
    def init_product(self, init_product, eps=0.0, noise=None):
        """Isometries carrying a product state: bottom node column 0 is
        phi_a (x) phi_b, upper node column 0 is e_0 (x) e_0; the other
        columns complete it by Gram-Schmidt of the unit vectors e_k, k = l +
        D_L r in order.  Optional dressing T += eps G / sqrt(D_L D_R) with the
        supplied complex normal stream G (node blocks in level-major order,
        l fastest).  Then QR-canonicalise toward the root and normalise."""
        tr = self.tree
        prod = torch.as_tensor(init_product, dtype=CDT)
        off = 0
        for v in range(tr.n_nodes):
            DL, DR, DP = tr.dims[v]
            if tr.is_bottom(v):
                a, b = tr.child_sites(v, 0)[0], tr.child_sites(v, 1)[0]
                c0 = torch.einsum("l,r->lr", prod[a], prod[b])
            else:
                c0 = torch.zeros(DL, DR, dtype=CDT)
                c0[0, 0] = 1.0
            cols = [c0.t().reshape(-1)]  # flat index l + DL*r
            for k in range(DL * DR):
                if len(cols) == DP:
                    break
                e = torch.zeros(DL * DR, dtype=CDT)
                e[k] = 1.0
                for c in cols:
                    coef = torch.vdot(c, e)
                    if coef != 0:
                        e = e - coef * c
                nrm = torch.linalg.vector_norm(e)
                if float(nrm) > COMPLETION_TOL:
                    cols.append(e / nrm)
            if len(cols) != DP:
                raise RuntimeError("isometry completion failed")
            M = torch.stack(cols, dim=1)                  # [(l + DL r), p]
            T = M.reshape(DR, DL, DP).permute(1, 0, 2).contiguous()
            if eps > 0:
                blk = torch.as_tensor(noise[off:off + DL * DR * DP], dtype=CDT)
                G = blk.reshape(DP, DR, DL).permute(2, 1, 0)
                T = T + (eps / math.sqrt(DL * DR)) * G
            off += DL * DR * DP
            self.T[v] = T
        self.canonicalise()

    def canonicalise(self):
        tr = self.tree
        for v in tr.postorder():
            if v == tr.root:
                self.T[v] = self.T[v] / torch.linalg.vector_norm(self.T[v])
                continue
            Q, R = qr_toward(self.T[v], 2)
            self.T[v] = Q
            u = tr.parent[v]
            self.T[u] = on_leg(tr.leg_in_parent(v), R, self.T[u])

    # -- Hamiltonian at the current time ----------------------------------
    def set_time(self, seg_edges, omega, delta, t, omega_x=None, omega_z=None):
        om, de, _ = pulse_at(seg_edges, torch.as_tensor(omega, dtype=RDT),
                             torch.as_tensor(delta, dtype=RDT), t)
        self.omega_t, self.delta_t = om.clone(), de.clone()
        zero = torch.zeros_like(torch.as_tensor(omega, dtype=RDT))
        ox, oz, _ = pulse_at(seg_edges, zero if omega_x is None else torch.as_tensor(omega_x, dtype=RDT),
                             zero if omega_z is None else torch.as_tensor(omega_z, dtype=RDT), t)
        self.omx_t, self.omz_t = ox.clone(), oz.clone()

    def h_local(self, site):
        om = self.omega_t[site]
        de = self.delta_t[site]
        h = (om / 2) * (self.X + self.leak_ratio * self.Lk) - de * self.n
        # single-qubit channels of Eq. (eq:ham) on {|0>, |1>}
        h = h + self.omx_t[site] * self.sx + self.omz_t[site] * self.sz
        if self.gamma != 0.0:
            # open system: decay out of |r> as the non-Hermitian term -i gamma |r><r|
            h = h - 1j * self.gamma * self.n
        return h

    # -- environments ----------------------------------------------------
    def child_env(self, v, side):
        """(H_block, {site: N_site}) of the child link `side` of node v, in
        that link's basis (physical basis for a leaf)."""
        tr = self.tree
        if tr.is_bottom(v):
            s = tr.child_sites(v, side)[0]
            return self.h_local(s), {s: self.n}
        e = self.up[tr.children[v][side]]
        return e["H"], e["N"]

    def parent_env(self, v):
        """(H_block, {site below v: W_site}) of v's parent link seen from
        above; the root's parent leg has dimension 1 and carries nothing."""
        tr = self.tree
        if v == tr.root:
            z = torch.zeros(1, 1, dtype=CDT)
            return z, {s: z for s in tr.sites_below(v)}
        e = self.down[v]
        return e["H"], e["W"]

    def A_op(self, i, NR):
        """sum_{j} V_ij N_j over the sites j of a right-hand environment."""
        acc = None
        for j, Nj in NR.items():
            t = float(self.V[i, j]) * Nj
            acc = t if acc is None else acc + t
        return acc

    def build_up(self, v):
        """Up environment of the link above v from its isometry Q = T[v]:
        H_up = Q^dag (H_L + H_R + sum_{i in L, j in R} V_ij n_i n_j) Q and
        N_i = Q^dag n_i Q for every site i below."""
        Q = self.T[v]
        HL, NL = self.child_env(v, 0)
        HR, NR = self.child_env(v, 1)
        X = on_L(HL, Q) + on_R(HR, Q)
        for i, Ni in NL.items():
            X = X + on_R(self.A_op(i, NR), on_L(Ni, Q))
        N = {}
        for i, Ni in NL.items():
            N[i] = proj(2, Q, on_L(Ni, Q))
        for j, Nj in NR.items():
            N[j] = proj(2, Q, on_R(Nj, Q))
        self.up[v] = dict(H=proj(2, Q, X), N=N)

    def build_down(self, c):
        """Down environment of the link above c from the isometry of its
        parent u canonical toward c: the block Hamiltonian of everything
        outside the subtree of c, and W_i = sum_{j outside} V_ij n_j for every
        site i inside."""
        tr = self.tree
        u = tr.parent[c]
        leg = tr.leg_in_parent(c)
        sib = 1 - leg
        Q = self.T[u]
        HS, NS = self.child_env(u, sib)
        HP, WP = self.parent_env(u)
        X = on_leg(sib, HS, Q) + on_P(HP, Q)
        for j, Nj in NS.items():
            X = X + on_P(WP[j], on_leg(sib, Nj, Q))
        W = {}
        for i in tr.sites_below(c):
            Y = on_leg(sib, self.A_op(i, NS), Q) + on_P(WP[i], Q)
            W[i] = proj(leg, Q, Y)
        self.down[c] = dict(H=proj(leg, Q, X), W=W)

    def rebuild_up(self):
        for v in self.tree.postorder():
            if v != self.tree.root:
                self.build_up(v)

    # -- effective Hamiltonians ------------------------------------------
    def heff(self, v):
        """T -> H_eff T at node v:  H_L + H_R + H_P (block terms), plus
        sum_{i in L} n_i (x) (A_i on R + W_i on P), plus sum_{j in R} n_j (x)
        W_j on P, where A_i = sum_{j in R} V_ij n_j."""
        HL, NL = self.child_env(v, 0)
        HR, NR = self.child_env(v, 1)
        HP, WP = self.parent_env(v)
        A = {i: self.A_op(i, NR) for i in NL}

        def apply(T):
            out = on_L(HL, T) + on_R(HR, T) + on_P(HP, T)
            for i, Ni in NL.items():
                Y = on_L(Ni, T)
                out = out + on_R(A[i], Y) + on_P(WP[i], Y)
            for j, Nj in NR.items():
                out = out + on_P(WP[j], on_R(Nj, T))
            return out
        return apply

    def keff(self, v):
        """C -> K_eff C on the link above v, C[below, above]:
        H_up C + C H_down^T + sum_i N_i C W_i^T."""
        Hb, Nb = self.up[v]["H"], self.up[v]["N"]
        Hd, Wd = self.down[v]["H"], self.down[v]["W"]

        def apply(C):
            out = Hb @ C + C @ Hd.t()
            for i, Ni in Nb.items():
                out = out + Ni @ C @ Wd[i].t()
            return out
        return apply

    def _expm(self, apply, x, tau):
        if self.gamma != 0.0:
            return arnoldi_expm(apply, x, tau, self.m)
        return lanczos_expm(apply, x, tau, self.m)

    def evolve_node(self, v, tau):
        out, info = self._expm(self.heff(v), self.T[v], tau)
        self.T[v] = out
        self.stats.append(("node", v, info["m"]))

    def evolve_bond(self, v, C, tau):
        out, info = self._expm(self.keff(v), C, -tau)
        self.stats.append(("bond", v, info["m"]))
        return out

    # -- sweeps ----------------------------------------------------------
    def _qr(self, T, leg):
        """Gauge-move QR (qr_toward) that also keeps the smallest R_kk seen
        since the last reset of qr_min: the conditioning of the step's gauge
        moves (a diagnostic; it changes no arithmetic)."""
        Q, R = qr_toward(T, leg)
        self.qr_min = min(self.qr_min, float(torch.diagonal(R).real.min().detach()))
        return Q, R

    def _visit_fwd(self, v, tau):
        tr = self.tree
        u, leg = tr.parent[v], tr.leg_in_parent(v)
        Q, R = self._qr(self.T[u], leg)
        self.T[u] = Q
        self.T[v] = on_P(R, self.T[v])          # absorb C = R^T below
        self.build_down(v)
        if not tr.is_bottom(v):
            for c in tr.children[v]:
                self._visit_fwd(c, tau)
        self.evolve_node(v, tau)
        Q, R = self._qr(self.T[v], 2)
        self.T[v] = Q
        self.build_up(v)
        C = self.evolve_bond(v, R, tau)
        self.T[u] = on_leg(leg, C, self.T[u])   # absorb C above

    def _visit_bwd(self, v, tau):
        tr = self.tree
        u, leg = tr.parent[v], tr.leg_in_parent(v)
        Q, R = self._qr(self.T[u], leg)
        self.T[u] = Q
        self.build_down(v)
        C = self.evolve_bond(v, R.t(), tau)
        self.T[v] = on_P(C.t(), self.T[v])      # T_v[.., k] = sum_a T_v[.., a] C[a, k]
        self.evolve_node(v, tau)
        if not tr.is_bottom(v):
            for c in reversed(tr.children[v]):
                self._visit_bwd(c, tau)
        Q, R = self._qr(self.T[v], 2)
        self.T[v] = Q
        self.build_up(v)
        self.T[u] = on_leg(leg, R, self.T[u])

    def sweep_fwd(self, tau):
        tr = self.tree
        for c in tr.children[tr.root] if not tr.is_bottom(tr.root) else []:
            self._visit_fwd(c, tau)
        self.evolve_node(tr.root, tau)

    def sweep_bwd(self, tau):
        tr = self.tree
        self.evolve_node(tr.root, tau)
        for c in reversed(tr.children[tr.root]) if not tr.is_bottom(tr.root) else []:
            self._visit_bwd(c, tau)

    # -- program events ----------------------------------------------------
    def apply_gate(self, site, U):
        b, side = self.tree.leaf_of_site(site)
        self.T[b] = on_leg(side, torch.as_tensor(U, dtype=CDT), self.T[b])

    # -- observables -------------------------------------------------------
    def norm2(self):
        return float(torch.linalg.vector_norm(self.T[self.tree.root]) ** 2)

    def rydberg_population(self):
        """sum_i <psi|n_i|psi> (unnormalised state): the total |r> population,
        whose time integral is the integrated time in the Rydberg state."""
        return sum(self.local_expectation(s, self.n).real for s in range(self.tree.N))

    def energy(self):
        """Re <psi|H|psi> with the centre at the root and current environments
        (the real part is the whole value for a Hermitian H)."""
        r = self.tree.root
        T = self.T[r]
        return float(torch.vdot(T.reshape(-1), self.heff(r)(T).reshape(-1)).real)

    def product_overlap(self, states):
        """<phi_1 (x) ... (x) phi_N | psi> for per-site states[site] (d,)."""
        return complex(self.product_overlap_t(states))

    def product_overlap_t(self, states):
        """The same overlap as a (differentiable) complex tensor."""
        tr = self.tree
        vec = {}
        st = torch.as_tensor(states, dtype=CDT)
        for v in range(tr.n_nodes):
            T = self.T[v]
            if tr.is_bottom(v):
                a, b = tr.child_sites(v, 0)[0], tr.child_sites(v, 1)[0]
                vl, vr = st[a].conj(), st[b].conj()
            else:
                vl, vr = vec[tr.children[v][0]], vec[tr.children[v][1]]
            vec[v] = torch.einsum("l,r,lrp->p", vl, vr, T)
        return vec[tr.root][0]

    def ghz_fidelity(self, target_sites):
        F, ov = self.ghz_fidelity_t(target_sites)
        return float(F), complex(ov)

    def ghz_fidelity_t(self, target_sites):
        """F = |<GHZ_S|psi>|^2 and the overlap, as tensors."""
        N, d = self.tree.N, self.d
        zero = torch.zeros(N, d, dtype=CDT)
        zero[:, 0] = 1.0
        one = zero.clone()
        for s in target_sites:
            one[int(s), 0] = 0.0
            one[int(s), 1] = 1.0
        ov = (self.product_overlap_t(zero) + self.product_overlap_t(one)) / math.sqrt(2.0)
        return ov.abs() ** 2, ov

    def local_expectation(self, site, op):
        """<psi|O_site|psi> by contracting the network with O on one leaf."""
        b, side = self.tree.leaf_of_site(site)
        other = OracleTTN.__new__(OracleTTN)
        other.tree = self.tree
        other.T = list(self.T)
        other.T[b] = on_leg(side, torch.as_tensor(op, dtype=CDT), self.T[b])
        return ttn_overlap(self, other)

    def dense_state(self):
        """Full state vector, site 0 the slowest index (small N only)."""
        tr = self.tree
        vec = {}
        for v in range(tr.n_nodes):
            T = self.T[v]
            if tr.is_bottom(v):
                vec[v] = (T, [tr.child_sites(v, 0)[0], tr.child_sites(v, 1)[0]])
            else:
                (A, sa), (B, sb) = vec[tr.children[v][0]], vec[tr.children[v][1]]
                Af = A.reshape(-1, A.shape[-1])
                Bf = B.reshape(-1, B.shape[-1])
                X = torch.einsum("al,br,lrp->abp", Af, Bf, T)
                vec[v] = (X.reshape(list(A.shape[:-1]) + list(B.shape[:-1]) + [T.shape[-1]]), sa + sb)
        X, sites = vec[tr.root]
        X = X[..., 0]
        perm = [sites.index(s) for s in range(tr.N)]
        return X.permute(*perm).reshape(-1)


def ttn_overlap(A: OracleTTN, B: OracleTTN) -> complex:
    """<psi_A|psi_B> by full bottom-up contraction (any gauge)."""
    tr = A.tree
    M = {}
    for v in range(tr.n_nodes):
        TA, TB = A.T[v], B.T[v]
        if tr.is_bottom(v):
            M[v] = torch.einsum("lrp,lrq->pq", TA.conj(), TB)
        else:
            ML, MR = M[tr.children[v][0]], M[tr.children[v][1]]
            M[v] = torch.einsum("lrp,lm,rs,msq->pq", TA.conj(), ML, MR, TB)
    return complex(M[tr.root][0, 0])


# ---------------------------------------------------------------------------
# driver
# ---------------------------------------------------------------------------

def build(w) -> OracleTTN:
    """Oracle state from a workload description (attribute access only)."""
    st = OracleTTN(w.n_sites, w.d, w.chi, w.pos_xy, w.leaf_order, w.c6, w.r_cut, w.leak_ratio,
                   w.krylov_dim, getattr(w, "gamma", 0.0))
    st.init_product(w.init_product, w.dress_eps, w.dress_noise)
    return st


def run(w, n_steps: Optional[int] = None, st: Optional[OracleTTN] = None, step0: int = 0,
        record=True, apply_final_events=True, omega=None, delta=None):
    """TDVP time evolution of the workload.  Step n: apply the gate events
    scheduled at n, freeze H at t_n + dt/2, rebuild the up environments,
    then S(dt/2) and S*(dt/2).  Events scheduled at the final step count are
    applied after the last step.  Returns the state and per-step records."""
    if st is None:
        st = build(w)
    n_steps = w.n_steps if n_steps is None else n_steps
    edges = torch.as_tensor(w.seg_edges, dtype=RDT)
    om = torch.as_tensor(w.omega, dtype=RDT) if omega is None else omega
    de = torch.as_tensor(w.delta, dtype=RDT) if delta is None else delta
    recs = []
    tau = w.dt / 2
    for n in range(step0, step0 + n_steps):
        for (k, s, U) in w.events:
            if k == n:
                st.apply_gate(s, U)
        st.set_time(edges, om, de, (n + 0.5) * w.dt, getattr(w, "omega_x", None), getattr(w, "omega_z", None))
        st.rebuild_up()
        st.qr_min = math.inf
        st.sweep_fwd(tau)
        st.sweep_bwd(tau)
        if record:
            rec = dict(step=n, norm2=st.norm2(), energy=st.energy(), min_r_diag=st.qr_min)
            if st.gamma != 0.0:
                rec["rydberg_population"] = st.rydberg_population()
            recs.append(rec)
    if apply_final_events:
        end = step0 + n_steps
        for (k, s, U) in w.events:
            if k == end:
                st.apply_gate(s, U)
    return st, recs


def fidelity_gradient(w, n_steps: Optional[int] = None, target_sites=None):
    """dF/dOmega and dF/dDelta of the discrete TDVP map: F = |<GHZ_S|psi_n>|^2
    after n_steps steps of run(), differentiated with respect to the pulse
    table (site-major [N][n_seg]) by reverse-mode automatic differentiation
    through every operation of the oracle (Lanczos, QR with the phase fix,
    environments, gates).  Returns (F, grad_omega, grad_delta) as numpy."""
    om = torch.tensor(w.omega, dtype=RDT, requires_grad=True)
    de = torch.tensor(w.delta, dtype=RDT, requires_grad=True)
    st, _ = run(w, n_steps=n_steps, record=False, omega=om, delta=de)
    F, _ = st.ghz_fidelity_t(w.target_sites if target_sites is None else target_sites)
    F.backward()
    return float(F.detach()), om.grad.detach().numpy().copy(), de.grad.detach().numpy().copy()
