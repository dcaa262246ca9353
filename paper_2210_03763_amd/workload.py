"""Seeded synthetic inputs for the TTN/TDVP Rydberg digital twin.

This module only *draws and lays out inputs*: lattice positions, the leaf
order of the binary tree, piecewise-constant pulse tables, exact local gate
events, the initial product state and the random dressing noise.  It holds
none of the method's arithmetic (no Hamiltonian, no tensor network, no
interaction potential); both the device library and the CPU oracle receive
these arrays and do every step of the method themselves.

Paper anchors (arXiv 2210.03763):
  * atoms on a 2D grid with positions (x_j, y_k) and lattice spacing a,
    Sec. "Modeling 88Sr quantum computers on two-dimensional grids";
  * leaves of the binary tree ordered along a Hilbert curve,
    Sec. "Tensor network simulations";
  * pulses switched per parallel layer; idle atoms carry zero drive,
    Sec. "Tensor network simulations";
  * CNOT built as Hadamard(target) . CZ . Hadamard(target), Sec. on the
    RydberGHZ compiler (gate decompositions);
  * repetition-code logical qubit = centre atom plus its four nearest
    neighbours, Sec. on parallel quantum error correction.

Synthetic stand-ins: the paper's time-optimal CZ pulses and compiled
circuits are not available, so CZ-type windows carry seeded random
Rabi/detuning values (Omega ~ U[0.5, 2], Delta ~ U[-1, 1]) of the same
layered shape.  Units are dimensionless (hbar = a = C6 = 1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# configuration
# ---------------------------------------------------------------------------

PREC_FP64 = 0
PREC_FP32 = 1
PREC_BF16X3 = 2


@dataclasses.dataclass
class Workload:
    """All inputs of one run, as plain numpy arrays."""

    name: str
    Lx: int
    Ly: int
    d: int
    chi: int
    n_steps: int
    dt: float
    krylov_dim: int
    precision: int
    c6: float
    r_cut: float            # <= 0 means all pairs
    leak_ratio: float       # amplitude of |leak><r| + h.c. relative to Omega/2 (d = 4)
    pos_xy: np.ndarray      # [N, 2] float64, site s at (x, y) with s = y * Lx + x
    leaf_order: np.ndarray  # [N] int32, leaf k of the tree holds site leaf_order[k]
    seg_edges: np.ndarray   # [S + 1] float64, segment s covers [edges[s], edges[s+1])
    omega: np.ndarray       # [N, S] float64
    delta: np.ndarray       # [N, S] float64
    events: List[Tuple[int, int, np.ndarray]]  # (step, site, U[d, d] complex128)
    init_product: np.ndarray  # [N, d] complex128, one normalised local state per site
    dress_eps: float
    dress_noise: Optional[np.ndarray]  # flat complex128 stream (see noise_len)
    target_sites: np.ndarray  # sites that carry the GHZ-type target; others are |0>
    seed: int
    ckpt_every: int = 0
    gamma: float = 0.0        # Rydberg decay rate of the open-system mode (0: closed system)
    # single-qubit drive on {|0>, |1>} of Eq. (eq:ham): Omega^x sigma^x + Omega^z sigma^z,
    # [N, S] on the same segments as omega/delta; None = zero
    omega_x: Optional[np.ndarray] = None
    omega_z: Optional[np.ndarray] = None
    update: int = 0           # 0 single-site TDVP, 1 two-site (two-tensor) update

    @property
    def n_sites(self) -> int:
        return self.Lx * self.Ly

    @property
    def n_seg(self) -> int:
        return int(self.omega.shape[1])

    def copy(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# lattice and leaf order
# ---------------------------------------------------------------------------

def square_positions(Lx: int, Ly: int) -> np.ndarray:
    """Site s = y * Lx + x sits at (x, y) in units of the spacing a."""
    pos = np.zeros((Lx * Ly, 2), dtype=np.float64)
    for y in range(Ly):
        for x in range(Lx):
            pos[y * Lx + x] = (x, y)
    return pos


def hex_positions(Lx: int, Ly: int) -> np.ndarray:
    """Hexagonal (triangular) arrangement with spacing a: site s = y * Lx + x
    sits at (x + (y mod 2)/2, y sqrt(3)/2), every atom has its nearest
    neighbours at distance a (Sec. on hexagonal lattices)."""
    pos = np.zeros((Lx * Ly, 2), dtype=np.float64)
    for y in range(Ly):
        for x in range(Lx):
            pos[y * Lx + x] = (x + 0.5 * (y % 2), y * math.sqrt(3.0) / 2.0)
    return pos


def hilbert_xy(k: int, idx: int) -> Tuple[int, int]:
    """Cell visited at position idx of the order-k Hilbert curve on a
    2^k x 2^k grid.  The curve starts at (0, 0) and ends at (2^k - 1, 0).

    Recursive construction: the four quadrants are visited lower-left,
    upper-left, upper-right, lower-right; the first quadrant holds the
    transposed order-(k-1) curve, the middle two hold translated copies and
    the last one the anti-transposed copy, so that consecutive cells are
    always lattice neighbours.
    """
    if k == 0:
        return 0, 0
    h = 1 << (k - 1)
    q, r = divmod(idx, h * h)
    x, y = hilbert_xy(k - 1, r)
    if q == 0:
        return y, x
    if q == 1:
        return x, y + h
    if q == 2:
        return x + h, y + h
    return 2 * h - 1 - y, h - 1 - x


def hilbert_leaf_order(Lx: int, Ly: int) -> np.ndarray:
    """Leaf order for an Lx x Ly lattice with Ly = 2^k and Lx a multiple of
    Ly: the lattice is cut into Lx/Ly squares side by side, each traversed by
    its own Hilbert curve, squares visited left to right."""
    k = int(round(math.log2(Ly)))
    if (1 << k) != Ly or Lx % Ly != 0:
        raise ValueError("need Ly = 2^k and Lx a multiple of Ly")
    order = []
    for blk in range(Lx // Ly):
        for i in range(Ly * Ly):
            x, y = hilbert_xy(k, i)
            order.append(y * Lx + (x + blk * Ly))
    return np.asarray(order, dtype=np.int32)


# ---------------------------------------------------------------------------
# local states and gates
# ---------------------------------------------------------------------------

def basis_state(d: int, k: int) -> np.ndarray:
    v = np.zeros(d, dtype=np.complex128)
    v[k] = 1.0
    return v


def plus_state(d: int) -> np.ndarray:
    v = np.zeros(d, dtype=np.complex128)
    v[0] = v[1] = 1.0 / math.sqrt(2.0)
    return v


def hadamard_gate(d: int) -> np.ndarray:
    """Hadamard on the qubit levels {|0>, |1>}; identity on |r> (and |leak>)."""
    u = np.eye(d, dtype=np.complex128)
    s = 1.0 / math.sqrt(2.0)
    u[0, 0] = s
    u[0, 1] = s
    u[1, 0] = s
    u[1, 1] = -s
    return u


# ---------------------------------------------------------------------------
# tree shape (only to size the dressing-noise stream)
# ---------------------------------------------------------------------------

def _capped_pow(d: int, e: int, cap: int) -> int:
    v = 1
    for _ in range(e):
        v *= d
        if v >= cap:
            return cap
    return v


def node_shapes(n_sites: int, d: int, chi: int) -> List[Tuple[int, int, int]]:
    """(D_left, D_right, D_parent) of every tree node, level by level from
    the bottom (level 0, two physical legs each) up to the root.  Used here
    only to size the noise stream; each consumer derives the shapes itself."""
    shapes = []
    n_lvl = int(round(math.log2(n_sites)))
    for lvl in range(n_lvl):
        n_nodes = n_sites >> (lvl + 1)
        s_child = 1 << lvl
        s_self = 1 << (lvl + 1)
        dc = min(_capped_pow(d, s_child, chi + 1), _capped_pow(d, n_sites - s_child, chi + 1), chi)
        if lvl == 0:
            dc = d
        dp = 1 if s_self == n_sites else min(
            _capped_pow(d, s_self, chi + 1), _capped_pow(d, n_sites - s_self, chi + 1), chi)
        shapes += [(dc, dc, dp)] * n_nodes
    return shapes


def noise_len(n_sites: int, d: int, chi: int) -> int:
    return int(sum(a * b * c for a, b, c in node_shapes(n_sites, d, chi)))


def _complex_normal(rng: np.random.Generator, n: int) -> np.ndarray:
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return (re + 1j * im) / math.sqrt(2.0)


# ---------------------------------------------------------------------------
# pulse programs
# ---------------------------------------------------------------------------

def _uniform_pulses(rng, n_sites, n_seg, active=None):
    om = rng.uniform(0.5, 2.0, size=(n_sites, n_seg))
    de = rng.uniform(-1.0, 1.0, size=(n_sites, n_seg))
    if active is not None:
        mask = np.zeros((n_sites, n_seg), dtype=bool)
        for s, sites in enumerate(active):
            mask[list(sites), s] = True
        om = np.where(mask, om, 0.0)
        de = np.where(mask, de, 0.0)
    return om, de


def ghz_layers(Lx: int, Ly: int, centre: int, n_layers_max: int, r_g: float, pos=None):
    """Greedy parallel GHZ schedule (a simple stand-in for the paper's
    compiler): layer by layer, disjoint (control in GHZ, target not yet in
    GHZ) nearest-neighbour pairs (distance a), targets ordered by distance to
    the centre then index; atoms of different pairs in one layer keep a
    distance >= r_g.  Returns the list of layers (each a list of (control,
    target)) or None if the lattice is not covered within n_layers_max
    layers.  pos: site positions (default: the square lattice)."""
    pos = square_positions(Lx, Ly) if pos is None else np.asarray(pos, dtype=np.float64)
    n = Lx * Ly
    cpos = pos[centre]

    def dist(a, b):
        return float(np.hypot(*(pos[a] - pos[b])))

    members = {centre}
    layers = []
    while len(members) < n:
        if len(layers) >= n_layers_max:
            return None
        cands = []
        for t in range(n):
            if t in members:
                continue
            for c in sorted(members):
                if abs(dist(c, t) - 1.0) < 1e-9:
                    cands.append((float(np.hypot(*(pos[t] - cpos))), t, c))
        cands.sort()
        used, chosen = set(), []
        for _, t, c in cands:
            if t in used or c in used:
                continue
            ok = True
            for (c2, t2) in chosen:
                for a in (c, t):
                    for b in (c2, t2):
                        if dist(a, b) < r_g - 1e-9:
                            ok = False
            if ok:
                chosen.append((c, t))
                used.add(t)
                used.add(c)
        if not chosen:
            return None
        layers.append(chosen)
        members |= {t for _, t in chosen}
    return layers


def hadamard_pulse_amplitude(n_steps: int, dt: float) -> float:
    """Omega^x = Omega^z = a for n_steps steps of dt gives
    exp(-i pi/2 (sigma^x + sigma^z)/sqrt 2) = -i H on {|0>, |1>}: a Hadamard
    as a square pulse of Eq. (eq:ham) (a global phase -i on the qubit
    levels, none on |r>)."""
    return math.pi / (2.0 * math.sqrt(2.0) * n_steps * dt)


def _layer_program(rng, Lx, Ly, d, n_steps, dt, layers, seg_per_layer, per_site_global=False,
                   n_global_seg=8, gates="exact", gate_steps=2, centre=None):
    """Pulse tables + gate events for a layered CZ-type program.

    Layer l covers steps [floor(n_steps*l/L), floor(n_steps*(l+1)/L)); its
    targets get an exact Hadamard at the first step of the layer and again
    at the step after its end.  Inside a layer only its atoms are driven,
    over `seg_per_layer` segments whose edges sit on step boundaries.
    With per_site_global, every site is driven on `n_global_seg` equal
    global segments instead (the gradient workload).

    gates="pulse": the Hadamards are square sigma^x/sigma^z pulses of
    gate_steps steps at the start and at the end of the layer window instead
    (the centre's first Hadamard joins the first window of layer 0), and the
    CZ-type drive fills the steps between them.  Returns (edges, omega,
    delta, events, omega_x, omega_z); the last two are None for exact gates."""
    n = Lx * Ly
    L = len(layers)
    had = hadamard_gate(d)
    events = []
    edges = [0.0]
    act = []
    hwin = []       # per segment: sites carrying a Hadamard pulse
    for l, pairs in enumerate(layers):
        s0 = (n_steps * l) // L
        s1 = (n_steps * (l + 1)) // L
        targets = {t for _, t in pairs}
        if gates == "pulse":
            if s1 - s0 < 2 * gate_steps + seg_per_layer:
                raise ValueError("layer window too short for its gate pulses")
            first = targets | ({centre} if (l == 0 and centre is not None) else set())
            lo, hi = s0 + gate_steps, s1 - gate_steps
            edges.append(lo * dt)
            act.append(set())
            hwin.append(first)
            for k in range(seg_per_layer):
                edges.append((lo + ((hi - lo) * (k + 1)) // seg_per_layer) * dt)
                act.append({a for pr in pairs for a in pr})
                hwin.append(set())
            edges.append(s1 * dt)
            act.append(set())
            hwin.append(targets)
            continue
        for t in targets:
            events.append((s0, t, had.copy()))
            events.append((s1, t, had.copy()))
        if not per_site_global:
            ln = s1 - s0
            for k in range(seg_per_layer):
                e = s0 + (ln * (k + 1)) // seg_per_layer
                if e > int(round(edges[-1] / dt)):
                    edges.append(e * dt)
                    act.append({a for pr in pairs for a in pr})
    if per_site_global:
        edges = [(n_steps * k // n_global_seg) * dt for k in range(n_global_seg + 1)]
        om, de = _uniform_pulses(rng, n, n_global_seg)
    else:
        om, de = _uniform_pulses(rng, n, len(act), act)
    if gates != "pulse":
        return np.asarray(edges), om, de, events, None, None
    a = hadamard_pulse_amplitude(gate_steps, dt)
    ox = np.zeros((n, len(act)))
    for k, sites in enumerate(hwin):
        ox[list(sites), k] = a
    return np.asarray(edges), om, de, events, ox, ox.copy()


# ---------------------------------------------------------------------------
# public constructors
# ---------------------------------------------------------------------------

def _base(name, Lx, Ly, d, chi, n_steps, dt, seed, precision=PREC_FP64, eps=1e-2):
    n = Lx * Ly
    return dict(name=name, Lx=Lx, Ly=Ly, d=d, chi=chi, n_steps=n_steps, dt=dt,
                krylov_dim=12, precision=precision, c6=1.0, r_cut=0.0,
                leak_ratio=0.05 if d == 4 else 0.0,
                pos_xy=square_positions(Lx, Ly),
                leaf_order=hilbert_leaf_order(Lx, Ly), seed=seed, dress_eps=eps,
                init_product=np.stack([basis_state(d, 0)] * n),
                target_sites=np.arange(n, dtype=np.int32))


def _finish(kw, rng):
    n = kw["Lx"] * kw["Ly"]
    if kw["dress_eps"] > 0:
        kw["dress_noise"] = _complex_normal(rng, noise_len(n, kw["d"], kw["chi"]))
    else:
        kw["dress_noise"] = None
    return Workload(**kw)


def make_random_drive(Lx, Ly, d, chi, n_steps, dt, n_seg, seed, plus_sites=(0,), eps=0.0,
                      precision=PREC_FP64, name="random-drive"):
    """Every site driven with Omega ~ U[0.5,2], Delta ~ U[-1,1] on n_seg
    equal segments over [0, n_steps*dt); initial |0...0> with |+> on the
    listed sites (the 4x4 chi=16 workload uses plus_sites=(0,))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kw = _base(name, Lx, Ly, d, chi, n_steps, dt, seed, precision, eps)
    n = Lx * Ly
    kw["seg_edges"] = np.asarray([(n_steps * k // n_seg) * dt for k in range(n_seg + 1)])
    kw["omega"], kw["delta"] = _uniform_pulses(rng, n, n_seg)
    kw["events"] = []
    prod = kw["init_product"].copy()
    for s in plus_sites:
        prod[s] = plus_state(d)
    kw["init_product"] = prod
    return _finish(kw, rng)


def make_ghz_program(Lx, Ly, d, chi, n_steps, dt, seed, n_layers=14, seg_per_layer=8,
                     per_site_global=False, eps=1e-2, precision=PREC_FP64, name="ghz",
                     lattice="square", gates="exact", gate_steps=2):
    """GHZ-preparation program: |0...0>, exact Hadamard on the centre atom
    at step 0, then CZ-type layers (Hadamard on targets around seeded
    random drive windows).  The widest inter-gate distance r_G in
    {2, sqrt 2, 1} whose greedy schedule covers the lattice within
    n_layers layers is used.  lattice="hex" places the atoms on the
    hexagonal arrangement (the tree keeps the index Hilbert order);
    gates="pulse" drives every Hadamard as a sigma^x/sigma^z square pulse of
    gate_steps steps through the TDVP instead of an exact gate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kw = _base(name, Lx, Ly, d, chi, n_steps, dt, seed, precision, eps)
    if lattice == "hex":
        kw["pos_xy"] = hex_positions(Lx, Ly)
    elif lattice != "square":
        raise ValueError(lattice)
    centre = (Ly // 2 - 1) * Lx + (Lx // 2 - 1)
    layers = None
    for r_g in (2.0, math.sqrt(2.0), 1.0):
        layers = ghz_layers(Lx, Ly, centre, n_layers, r_g, pos=kw["pos_xy"])
        if layers is not None:
            break
    if layers is None:
        raise RuntimeError("no GHZ schedule fits")
    edges, om, de, ev, ox, oz = _layer_program(rng, Lx, Ly, d, n_steps, dt, layers, seg_per_layer,
                                               per_site_global, gates=gates, gate_steps=gate_steps,
                                               centre=centre)
    kw.update(seg_edges=edges, omega=om, delta=de, omega_x=ox, omega_z=oz)
    kw["events"] = ([(0, centre, hadamard_gate(d))] if gates != "pulse" else []) + ev
    return _finish(kw, rng)


def make_repcode_program(Lx, Ly, d, chi, n_steps, dt, seed, eps=1e-2, precision=PREC_FP64,
                         seg_per_layer=8, name="repcode"):
    """Five-qubit repetition code (centre atom + its four nearest
    neighbours) prepared by four serial CZ-type layers; all other atoms idle
    in |0>.  Target (|00000> + |11111>)/sqrt 2 on the five code atoms."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kw = _base(name, Lx, Ly, d, chi, n_steps, dt, seed, precision, eps)
    cx, cy = Lx // 2 - 1, Ly // 2 - 1
    centre = cy * Lx + cx
    nbrs = [cy * Lx + cx + 1, (cy + 1) * Lx + cx, cy * Lx + cx - 1, (cy - 1) * Lx + cx]
    layers = [[(centre, t)] for t in nbrs]
    edges, om, de, ev, _, _ = _layer_program(rng, Lx, Ly, d, n_steps, dt, layers, seg_per_layer)
    kw.update(seg_edges=edges, omega=om, delta=de)
    kw["events"] = [(0, centre, hadamard_gate(d))] + ev
    kw["target_sites"] = np.asarray([centre] + nbrs, dtype=np.int32)
    return _finish(kw, rng)


# The five benchmark workloads (seed 2210037630 + k for the k-th).
def config(name: str, **over) -> Workload:
    seed0 = 2210037630
    if name == "c1":      # 4x4, d=3, chi=16, 20 steps, |+> on site 0, undressed
        w = make_random_drive(4, 4, 3, 16, 20, 0.01, 4, seed0 + 1, plus_sites=(0,), eps=0.0,
                              name="4x4 d3 chi16 random drive, |+> on site 0")
    elif name == "c1-ent":  # same drive, |+> on every site, dressed
        w = make_random_drive(4, 4, 3, 16, 20, 0.01, 4, seed0 + 1, plus_sites=tuple(range(16)),
                              eps=1e-2, name="4x4 d3 chi16 random drive, |+> on all sites")
    elif name == "c2":
        w = make_ghz_program(8, 8, 3, 64, 200, 0.005, seed0 + 2,
                             name="8x8 d3 chi64 GHZ program (FP64)")
    elif name == "c3":
        w = make_ghz_program(8, 8, 4, 128, 200, 0.005, seed0 + 3, precision=PREC_FP32,
                             name="8x8 d4 chi128 GHZ program (mixed)")
    elif name == "c4":
        w = make_ghz_program(8, 8, 3, 64, 200, 0.005, seed0 + 4, per_site_global=True,
                             name="8x8 d3 chi64 GHZ gates, 64x8 per-site segments")
        w.ckpt_every = 10
    elif name == "hex-pulse":   # 8x8 hexagonal, Hadamards as sigma^x/sigma^z square pulses
        w = make_ghz_program(8, 8, 4, 128, 200, 0.005, seed0 + 6, precision=PREC_FP32, lattice="hex",
                             gates="pulse", gate_steps=2,
                             name="8x8 hexagonal d4 chi128 GHZ program, pulse-driven gates (mixed)")
    elif name == "c5":
        w = make_repcode_program(8, 8, 4, 256, 400, 0.0025, seed0 + 5, precision=PREC_FP32,
                                 name="8x8 d4 chi256 repetition code (mixed)")
    else:
        raise KeyError(name)
    for k, v in over.items():
        setattr(w, k, v)
    return w
