"""Dense state-vector reference: the plain definition of the evolution.

TEST INFRASTRUCTURE (same import rule as ttn_oracle).  For small lattices
the TDVP oracle is pinned against psi_{n+1} = exp(-i H(t_n + dt/2) dt) psi_n
with the full Hamiltonian of Eq. (eq:ham)/(eq:c6) (read as in ttn_oracle:
Omega/2 on |1><r| + h.c., -Delta |r><r|, optional leak coupling, the
single-qubit channels Omega^x sigma^x + Omega^z sigma^z, positive
C6/d^6 over pairs i < j, and -i gamma |r><r| per site for the open system of
Eq. (eq:hoqs)) built as a sparse matrix on the product basis
(site 0 the slowest index), and evolved with scipy's expm_multiply.  At
maximal bond dimension single-site TDVP reproduces this exactly (the
exactness of projector-splitting integrators, Lubich, Oseledets and
Vandereycken 2015).  fidelity_gradient differentiates this map exactly
(Frechet derivative of each step's exponential); it pins the gradient of the
TDVP oracle at maximal bond dimension.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _ops(d):
    X = np.zeros((d, d), complex)
    n = np.zeros((d, d), complex)
    Lk = np.zeros((d, d), complex)
    X[1, 2] = X[2, 1] = 1
    n[2, 2] = 1
    if d >= 4:
        Lk[3, 2] = Lk[2, 3] = 1
    return X, n, Lk


def _embed(op, site, N, d):
    out = sp.identity(1, dtype=complex, format="csr")
    for s in range(N):
        out = sp.kron(out, sp.csr_matrix(op) if s == site else sp.identity(d, dtype=complex),
                      format="csr")
    return out


def hamiltonian(pos, d, omega_t, delta_t, c6=1.0, r_cut=0.0, leak_ratio=0.0, gamma=0.0, omx_t=None,
                omz_t=None):
    N = len(pos)
    X, n, Lk = _ops(d)
    sx = np.zeros((d, d), complex)
    sz = np.zeros((d, d), complex)
    sx[0, 1] = sx[1, 0] = 1
    sz[0, 0], sz[1, 1] = 1, -1
    H = sp.csr_matrix((d ** N, d ** N), dtype=complex)
    nsite = [_embed(n, s, N, d) for s in range(N)]
    for s in range(N):
        hl = omega_t[s] / 2 * (X + leak_ratio * Lk) - (delta_t[s] + 1j * gamma) * n
        if omx_t is not None:
            hl = hl + omx_t[s] * sx + omz_t[s] * sz
        if np.any(hl != 0):
            H = H + _embed(hl, s, N, d)
    for i in range(N):
        for j in range(i + 1, N):
            dist = math.hypot(pos[i][0] - pos[j][0], pos[i][1] - pos[j][1])
            if r_cut > 0 and dist > r_cut:
                continue
            H = H + (c6 / dist ** 6) * (nsite[i] @ nsite[j])
    return H


def product_vector(states):
    v = np.ones(1, complex)
    for s in states:
        v = np.kron(v, np.asarray(s, complex))
    return v


def apply_local(psi, U, site, N, d):
    t = psi.reshape([d] * N)
    t = np.moveaxis(np.tensordot(U, t, axes=([1], [site])), 0, site)
    return t.reshape(-1)


def pulse_index(edges, t):
    for s in range(len(edges) - 1):
        if edges[s] <= t < edges[s + 1]:
            return s
    return -1


def run(w, psi0, n_steps=None, step0=0, apply_final_events=True):
    """Evolve psi0 (site 0 slowest) with the workload's program."""
    N, d = w.n_sites, w.d
    n_steps = w.n_steps if n_steps is None else n_steps
    psi = np.asarray(psi0, complex).copy()
    for n in range(step0, step0 + n_steps):
        for (k, s, U) in w.events:
            if k == n:
                psi = apply_local(psi, U, s, N, d)
        t = (n + 0.5) * w.dt
        sidx = pulse_index(w.seg_edges, t)
        om = w.omega[:, sidx] if sidx >= 0 else np.zeros(N)
        de = w.delta[:, sidx] if sidx >= 0 else np.zeros(N)
        ox = oz = None
        if getattr(w, "omega_x", None) is not None:
            ox = w.omega_x[:, sidx] if sidx >= 0 else np.zeros(N)
            oz = w.omega_z[:, sidx] if sidx >= 0 else np.zeros(N)
        H = hamiltonian(w.pos_xy, d, om, de, w.c6, w.r_cut, w.leak_ratio, getattr(w, "gamma", 0.0), ox, oz)
        psi = spla.expm_multiply(-1j * w.dt * H, psi)
    if apply_final_events:
        for (k, s, U) in w.events:
            if k == step0 + n_steps:
                psi = apply_local(psi, U, s, N, d)
    return psi


def fidelity_gradient(w, psi0, target_sites=None):
    """F = |<GHZ_S|psi_final>|^2 of run() and its exact derivative with respect
    to every entry of the pulse tables (site-major [N][n_seg]).

    Each step is U_n = exp(A_n), A_n = -i dt H(t_n + dt/2), and H depends
    linearly on the pulse values of the segment the step samples, so
    dU_n = L(A_n, -i dt dH) with L the Frechet derivative of the matrix
    exponential (scipy.linalg.expm_frechet).  With the adjoint state
    lambda_{n+1} = (everything after U_n)^dag |GHZ_S>,
    dF = 2 Re(conj(o) sum_n <lambda_{n+1}| dU_n |psi_n>), o = <GHZ_S|psi_final>.
    Returns (F, grad_omega, grad_delta)."""
    import scipy.linalg as sla
    N, d = w.n_sites, w.d
    X, n, Lk = _ops(d)
    tsites = list(range(N)) if target_sites is None else [int(s) for s in target_sites]
    if target_sites is None and getattr(w, "target_sites", None) is not None:
        tsites = [int(s) for s in w.target_sites]
    zero = np.zeros((N, d), complex)
    zero[:, 0] = 1
    one = zero.copy()
    for s in tsites:
        one[s] = 0
        one[s, 1] = 1
    g = (product_vector(zero) + product_vector(one)) / math.sqrt(2.0)
    # forward, keeping the state just before each exponential
    psi = np.asarray(psi0, complex).copy()
    pre, gens, segs = [], [], []
    for k in range(w.n_steps):
        for (kk, s, U) in w.events:
            if kk == k:
                psi = apply_local(psi, U, s, N, d)
        sidx = pulse_index(w.seg_edges, (k + 0.5) * w.dt)
        om = w.omega[:, sidx] if sidx >= 0 else np.zeros(N)
        de = w.delta[:, sidx] if sidx >= 0 else np.zeros(N)
        A = (-1j * w.dt) * hamiltonian(w.pos_xy, d, om, de, w.c6, w.r_cut, w.leak_ratio).toarray()
        pre.append(psi.copy())
        gens.append(A)
        segs.append(sidx)
        psi = sla.expm(A) @ psi
    for (kk, s, U) in w.events:
        if kk == w.n_steps:
            psi = apply_local(psi, U, s, N, d)
    o = np.vdot(g, psi)
    F = abs(o) ** 2
    # adjoint sweep
    lam = g.copy()
    for (kk, s, U) in w.events:
        if kk == w.n_steps:
            lam = apply_local(lam, np.conj(U).T, s, N, d)
    gO = np.zeros_like(w.omega, dtype=float)
    gD = np.zeros_like(w.delta, dtype=float)
    dOm = [_embed((X + w.leak_ratio * Lk) / 2, s, N, d).toarray() for s in range(N)]
    dDe = [-_embed(n, s, N, d).toarray() for s in range(N)]
    for k in reversed(range(w.n_steps)):
        A, sidx = gens[k], segs[k]
        if sidx >= 0:
            for s in range(N):
                for dH, out in ((dOm[s], gO), (dDe[s], gD)):
                    _, L = sla.expm_frechet(A, (-1j * w.dt) * dH)
                    out[s, sidx] += 2.0 * (np.conj(o) * np.vdot(lam, L @ pre[k])).real
        lam = sla.expm(A).conj().T @ lam
        for (kk, s, U) in w.events:
            if kk == k:
                lam = apply_local(lam, np.conj(U).T, s, N, d)
    return F, gO, gD
