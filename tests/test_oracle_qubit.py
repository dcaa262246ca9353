"""Pins of the single-qubit drive channels of Eq. (eq:ham) (Omega^x sigma^x
+ Omega^z sigma^z on {|0>, |1>}) and of non-square lattices.

  * closed forms at maximal chi: a sigma^x pulse of area theta takes |0> to
    cos theta |0> - i sin theta |1>; a sigma^z pulse gives |+> the phases
    e^{-i theta} / e^{+i theta}; equal sigma^x and sigma^z pulses of area
    pi/(2 sqrt 2) each give -i H |0> (the Hadamard as a square pulse);
  * a GHZ program on a hexagonal lattice whose Hadamards are square pulses
    through the TDVP equals the dense evolution at maximal chi;
  * the hexagonal arrangement puts every atom's nearest neighbours at
    distance a (six in the bulk).
"""
import math

import numpy as np
import pytest

from oracle import dense as D
from oracle import ttn_oracle as O
from paper_2210_03763_amd import workload as W


def _two_atoms(ox, oz, init, steps=10, dt=0.01):
    w = W.make_random_drive(2, 1, 3, 9, steps, dt, 1, seed=3, plus_sites=(), eps=0.0)
    z = np.zeros_like(w.omega)
    w = w.copy(omega=z, delta=z, omega_x=np.array([[ox], [0.0]]), omega_z=np.array([[oz], [0.0]]),
               init_product=np.stack([init, W.basis_state(3, 0)]))
    st, _ = O.run(w)
    return st.dense_state().numpy().reshape(3, 3)[:, 0], w


def test_sigma_x_rotation_closed_form():
    theta = 0.7
    psi, w = _two_atoms(theta / (10 * 0.01), 0.0, W.basis_state(3, 0))
    ref = np.array([math.cos(theta), -1j * math.sin(theta), 0.0])
    assert np.abs(psi - ref).max() < 1e-12


def test_sigma_z_phase_closed_form():
    theta = 0.9
    psi, w = _two_atoms(0.0, theta / (10 * 0.01), W.plus_state(3))
    ref = np.array([np.exp(-1j * theta), np.exp(1j * theta), 0.0]) / math.sqrt(2)
    assert np.abs(psi - ref).max() < 1e-12


def test_hadamard_as_square_pulse():
    a = W.hadamard_pulse_amplitude(10, 0.01)
    psi, w = _two_atoms(a, a, W.basis_state(3, 0))
    ref = -1j * np.array([1.0, 1.0, 0.0]) / math.sqrt(2)
    assert np.abs(psi - ref).max() < 1e-12


def test_hex_pulse_program_maximal_chi_equals_dense():
    w = W.make_ghz_program(2, 2, 3, 9, 24, 0.02, seed=17, n_layers=3, seg_per_layer=2, eps=0.05,
                           lattice="hex", gates="pulse", gate_steps=2)
    assert w.omega_x is not None and np.count_nonzero(w.omega_x) > 0 and not w.events
    st = O.build(w)
    psi0 = st.dense_state().numpy()
    st, recs = O.run(w, st=st)
    ref = D.run(w, psi0)
    assert np.abs(st.dense_state().numpy() - ref).max() < 1e-10
    # the pulse program differs from the same program with the qubit drive off
    off = D.run(w.copy(omega_x=None, omega_z=None), psi0)
    assert np.abs(off - ref).max() > 1e-2


def test_hex_positions_nearest_neighbours():
    pos = W.hex_positions(8, 8)
    dist = np.hypot(*(pos[:, None, :] - pos[None, :, :]).transpose(2, 0, 1))
    np.fill_diagonal(dist, np.inf)
    assert abs(dist.min() - 1.0) < 1e-12
    nn = (np.abs(dist - 1.0) < 1e-9).sum(axis=1)
    bulk = [y * 8 + x for y in range(1, 7) for x in range(1, 7)]
    assert (nn[bulk] == 6).all()
