"""Pins of the two-site TDVP oracle (oracle/two_site.py) on the CPU.

* Maximal chi: every two-site and single-site space of the network is then
  the whole space, so the integrator is exact; from an undressed product
  state (the padded isometries carry exact zeros, which the SVD split, unlike
  a Cholesky QR, accepts) it must reproduce the dense state-vector evolution.
* The split is the best rank-k approximation (Eckart-Young), checked against
  an eigendecomposition of Theta Theta^dag rather than the SVD it uses.
* A constant Hamiltonian conserves the energy at maximal chi.
* At truncated chi the state stays normalised, the recorded discarded
  weights are what the splits dropped, and the state stays close to the
  dense one for a short evolution.
"""
import numpy as np
import pytest
import torch

from oracle import dense as D
from oracle import ttn_oracle as O
from oracle import two_site as TS
from paper_2210_03763_amd import workload as W


def _two_site_run(w, cutoff=0.0):
    st = TS.build(w, cutoff=cutoff)
    psi0 = st.dense_state().numpy()
    st, recs = O.run(w, st=st)
    return st, recs, psi0


@pytest.mark.parametrize("Lx,Ly,chi", [(2, 2, 9), (4, 2, 81)])
def test_maximal_chi_matches_dense_from_undressed_product_state(Lx, Ly, chi):
    w = W.make_random_drive(Lx, Ly, 3, chi, 6, 0.05, 3, seed=7, plus_sites=(0, 1, 2, 3), eps=0.0)
    st, recs, psi0 = _two_site_run(w)
    ref = D.run(w, psi0)
    got = st.dense_state().numpy()
    assert np.abs(got - ref).max() < 1e-9
    assert max(st.discarded) < 1e-20   # nothing of weight is dropped at maximal chi
    # the product state really is undressed: a single non-zero amplitude pattern
    assert abs(np.linalg.norm(psi0) - 1.0) < 1e-14


def test_split_is_the_best_rank_k_approximation():
    g = torch.Generator().manual_seed(3)
    Theta = torch.randn(3, 4, 5, 2, dtype=torch.complex128, generator=g)
    Theta = Theta / torch.linalg.vector_norm(Theta)
    M = Theta.reshape(12, 10)
    for k in (1, 3, 7, 10):
        U, S, Vh, kept, disc = TS.truncated_split(Theta, k)
        assert kept == k
        # undo the norm-restoring rescale of the kept values
        norm_kept = float(torch.linalg.vector_norm(S))
        Mk = (U * (S / norm_kept * (1.0 - disc) ** 0.5).to(torch.complex128)) @ Vh
        # best rank-k approximation from the top-k eigenvectors of M M^dag
        lam, P = torch.linalg.eigh(M @ M.conj().t())
        Pk = P[:, -k:]
        Mref = Pk @ (Pk.conj().t() @ M)
        assert float(torch.linalg.matrix_norm(Mk - Mref)) < 1e-12
        assert abs(disc - (1.0 - float(lam[-k:].sum()))) < 1e-12
        # orthonormal factors and the rescaled norm
        assert float(torch.linalg.matrix_norm(U.conj().t() @ U - torch.eye(k, dtype=U.dtype))) < 1e-12
        assert float(torch.linalg.matrix_norm(Vh @ Vh.conj().t() - torch.eye(k, dtype=Vh.dtype))) < 1e-12
        assert abs(norm_kept - 1.0) < 1e-12


def test_constant_hamiltonian_conserves_energy_at_maximal_chi():
    w = W.make_random_drive(4, 2, 3, 81, 5, 0.05, 1, seed=9, plus_sites=(0, 2, 5), eps=0.0)
    st = TS.build(w)
    st.set_time(torch.as_tensor(w.seg_edges), torch.as_tensor(w.omega), torch.as_tensor(w.delta), 0.5 * w.dt)
    st.rebuild_up()
    e0 = st.energy()
    st, recs = O.run(w, st=st)
    assert all(abs(r["energy"] - e0) < 1e-10 for r in recs)


def test_truncated_chi_keeps_the_norm_and_records_the_discarded_weight():
    w = W.make_random_drive(4, 2, 3, 2, 10, 0.1, 3, seed=7, plus_sites=(0, 1, 2, 3), eps=0.0)
    st, recs, psi0 = _two_site_run(w)
    assert all(abs(r["norm2"] - 1.0) < 1e-12 for r in recs)
    disc = np.asarray(st.discarded)
    assert (disc >= 0).all() and (disc <= 1).all()
    assert disc.max() > 1e-12        # chi = 2 does truncate here
    assert disc.max() < 1e-4         # and only a little of the weight per split
    ref = D.run(w, psi0)
    fid = abs(np.vdot(ref, st.dense_state().numpy())) ** 2
    assert 0.999 < fid < 1.0
