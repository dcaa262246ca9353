"""Thin ctypes binding of libttn.so (include/ttn.h).

Argument marshalling only: every step of the TDVP path runs in the HIP
kernels of the library.  PyTorch provides the device workspace and the
stream.  The library must be built (paper_2210_03763_amd.build); nothing
here falls back to another implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttn.so")

TTN_OK, TTN_EINVAL, TTN_ENOMEM, TTN_EDEVICE, TTN_ENUMERIC, TTN_ESTATE, TTN_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
PREC_FP64, PREC_FP32, PREC_BF16X3 = 0, 1, 2
UPDATE_ONE_SITE, UPDATE_TWO_SITE = 0, 1

_ERRNAMES = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENUMERIC", -5: "ESTATE", -6: "ENOTSUP"}


class TTNError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("n_sites", C.c_int32), ("d", C.c_int32), ("chi", C.c_int32),
                ("krylov_dim", C.c_int32), ("precision", C.c_int32), ("update", C.c_int32),
                ("c6", C.c_double), ("r_cut", C.c_double), ("leak_ratio", C.c_double),
                ("pos_xy", C.POINTER(C.c_double)), ("leaf_order", C.POINTER(C.c_int32)),
                ("init_product", C.POINTER(C.c_double)), ("dress_eps", C.c_double),
                ("dress_noise", C.POINTER(C.c_double)), ("dress_noise_len", C.c_int64),
                ("gamma", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("norm2", C.c_double), ("energy", C.c_double), ("min_r_diag", C.c_double),
                ("min_krylov", C.c_int32), ("reserved", C.c_int32), ("max_discarded", C.c_double)]


class KernelProf(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("flops", C.c_double)]


class VecProf(C.Structure):
    _fields_ = [("calls", C.c_int64), ("ms", C.c_double), ("bytes", C.c_double)]


class Profile(C.Structure):
    _fields_ = [("gemm_f32", KernelProf), ("gemm_f64", KernelProf), ("heff", KernelProf),
                ("matvecs", C.c_int64), ("gemm_bf16x3", KernelProf), ("lanczos", VecProf),
                ("lanczos_large", VecProf)]


class LaunchRec(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("prec", C.c_int32), ("heff", C.c_int32), ("splits", C.c_int32),
                ("matvec", C.c_int32), ("reserved", C.c_int32), ("flops", C.c_double), ("ms", C.c_double)]


_lib = None


def lib():
    """Load libttn.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname; importing it
        # first makes this library bind to that runtime instead of loading a
        # second one from the system path (two runtimes cannot share a device)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: run paper_2210_03763_amd.build.build() first")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        DP = C.POINTER(C.c_double)
        IP = C.POINTER(C.c_int32)
        sig = {
            "ttn_workspace_query": (C.c_int, [C.POINTER(Config), C.POINTER(C.c_size_t)]),
            "ttn_init": (C.c_int, [C.POINTER(Config), P, C.c_size_t, P, C.POINTER(P)]),
            "ttn_set_pulses": (C.c_int, [P, I32, DP, DP, DP, I32, IP, IP, DP]),
            "ttn_set_qubit_pulses": (C.c_int, [P, DP, DP]),
            "ttn_tdvp_step": (C.c_int, [P, D, I32, C.POINTER(StepStats)]),
            "ttn_fidelity": (C.c_int, [P, I32, IP, DP, DP]),
            "ttn_observables": (C.c_int, [P, DP, DP]),
            "ttn_local_expectation": (C.c_int, [P, I32, DP, DP]),
            "ttn_rydberg_population": (C.c_int, [P, DP]),
            "ttn_overlap": (C.c_int, [P, P, DP]),
            "ttn_export_state": (I64, [P, DP, I64]),
            "ttn_set_graphs": (C.c_int, [P, I32]),
            "ttn_sample_query": (C.c_int, [P, I32, C.POINTER(C.c_size_t)]),
            "ttn_sample": (C.c_int, [P, I64, C.c_uint64, I64, P, C.c_size_t, C.POINTER(C.c_uint8), DP]),
            "ttn_adjoint_query": (C.c_int, [C.POINTER(Config), I32, I32, C.POINTER(C.c_size_t)]),
            "ttn_record_begin": (C.c_int, [P, I32, I32, P, C.c_size_t]),
            "ttn_backward": (C.c_int, [P, I32, IP, D, DP, DP]),
            "ttn_profile_begin": (C.c_int, [P]),
            "ttn_profile_begin_untimed": (C.c_int, [P]),
            "ttn_profile_end": (C.c_int, [P, C.POINTER(Profile)]),
            "ttn_profile_launches": (I64, [P, C.POINTER(LaunchRec), I64]),
            "ttn_destroy": (C.c_int, [P]),
            "ttn_last_error": (C.c_char_p, [P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _complex_interleaved(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    return a.view(np.float64).reshape(-1).copy()


def make_config(w, keep: list) -> Config:
    """ttn_config from a workload description; `keep` holds the arrays alive."""
    pos = np.ascontiguousarray(w.pos_xy, dtype=np.float64).reshape(-1)
    order = np.ascontiguousarray(w.leaf_order, dtype=np.int32)
    prod = _complex_interleaved(w.init_product)
    noise = _complex_interleaved(w.dress_noise) if (w.dress_eps > 0 and w.dress_noise is not None) else None
    keep += [pos, order, prod, noise]
    cfg = Config()
    cfg.n_sites = w.n_sites
    cfg.d = w.d
    cfg.chi = w.chi
    cfg.krylov_dim = w.krylov_dim
    cfg.precision = w.precision
    cfg.update = int(getattr(w, "update", 0))
    cfg.c6 = w.c6
    cfg.r_cut = w.r_cut
    cfg.leak_ratio = w.leak_ratio
    cfg.pos_xy = _dptr(pos)
    cfg.leaf_order = _iptr(order)
    cfg.init_product = _dptr(prod)
    cfg.dress_eps = w.dress_eps
    cfg.dress_noise = _dptr(noise) if noise is not None else C.POINTER(C.c_double)()
    cfg.dress_noise_len = 0 if noise is None else noise.size // 2
    cfg.gamma = float(getattr(w, "gamma", 0.0))
    return cfg


def workspace_bytes(w) -> int:
    keep: list = []
    cfg = make_config(w, keep)
    out = C.c_size_t(0)
    rc = lib().ttn_workspace_query(C.byref(cfg), C.byref(out))
    if rc != TTN_OK:
        raise TTNError(rc, "workspace query failed")
    return int(out.value)


class TTN:
    """One TTN state on the current CUDA (HIP) device."""

    def __init__(self, w, device=None, stream=None):
        import torch
        self._keep: list = []
        self.w = w
        self.device = torch.device("cuda") if device is None else torch.device(device)
        cfg = make_config(w, self._keep)
        nbytes = C.c_size_t(0)
        self._check(lib().ttn_workspace_query(C.byref(cfg), C.byref(nbytes)), None)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        h = C.c_void_p()
        rc = lib().ttn_init(C.byref(cfg), C.c_void_p(self.workspace.data_ptr()), nbytes,
                            C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self._check(rc, None)
        self.h = h
        self.set_pulses(w.seg_edges, w.omega, w.delta, w.events)
        if getattr(w, "omega_x", None) is not None or getattr(w, "omega_z", None) is not None:
            self.set_qubit_pulses(w.omega_x, w.omega_z)

    def _check(self, rc, h):
        if rc < 0:
            raise TTNError(rc, lib().ttn_last_error(h).decode())
        return rc

    def set_pulses(self, edges, omega, delta, events: Sequence = ()):
        edges = np.ascontiguousarray(edges, dtype=np.float64)
        om = np.ascontiguousarray(omega, dtype=np.float64)
        de = np.ascontiguousarray(delta, dtype=np.float64)
        steps = np.ascontiguousarray([e[0] for e in events], dtype=np.int32)
        sites = np.ascontiguousarray([e[1] for e in events], dtype=np.int32)
        us = (_complex_interleaved(np.stack([e[2] for e in events])) if len(events)
              else np.zeros(2, np.float64))
        self._pulses = (edges, om, de, steps, sites, us)
        rc = lib().ttn_set_pulses(self.h, int(om.shape[1]) if om.ndim == 2 else 0, _dptr(edges), _dptr(om),
                                  _dptr(de), len(events), _iptr(steps), _iptr(sites), _dptr(us))
        self._check(rc, self.h)

    def set_qubit_pulses(self, omega_x, omega_z):
        """Omega^x / Omega^z tables [N][n_seg] on the current segments (None = zero)."""
        ox = None if omega_x is None else np.ascontiguousarray(omega_x, dtype=np.float64)
        oz = None if omega_z is None else np.ascontiguousarray(omega_z, dtype=np.float64)
        self._qubit = (ox, oz)
        null = C.POINTER(C.c_double)()
        rc = lib().ttn_set_qubit_pulses(self.h, null if ox is None else _dptr(ox), null if oz is None else _dptr(oz))
        self._check(rc, self.h)

    def step(self, n_steps: int, dt: Optional[float] = None, stats: bool = False):
        dt = self.w.dt if dt is None else dt
        arr = (StepStats * max(1, n_steps))() if stats else None
        rc = lib().ttn_tdvp_step(self.h, float(dt), int(n_steps), arr)
        self._check(rc, self.h)
        if stats:
            return [dict(norm2=a.norm2, energy=a.energy, min_r_diag=a.min_r_diag,
                         min_krylov=a.min_krylov, max_discarded=a.max_discarded) for a in arr[:n_steps]]
        return None

    def fidelity(self, target_sites=None):
        ts = np.ascontiguousarray(self.w.target_sites if target_sites is None else target_sites,
                                  dtype=np.int32)
        F = C.c_double(0)
        ov = np.zeros(2)
        self._check(lib().ttn_fidelity(self.h, len(ts), _iptr(ts), C.byref(F), _dptr(ov)), self.h)
        return F.value, complex(ov[0], ov[1])

    def observables(self):
        n2, e = C.c_double(0), C.c_double(0)
        self._check(lib().ttn_observables(self.h, C.byref(n2), C.byref(e)), self.h)
        return n2.value, e.value

    def rydberg_population(self) -> float:
        """sum_i <psi|n_i|psi> of the (unnormalised) current state."""
        p = C.c_double(0)
        self._check(lib().ttn_rydberg_population(self.h, C.byref(p)), self.h)
        return p.value

    def local_expectation(self, site: int, op) -> complex:
        o = _complex_interleaved(op)
        out = np.zeros(2)
        self._check(lib().ttn_local_expectation(self.h, int(site), _dptr(o), _dptr(out)), self.h)
        return complex(out[0], out[1])

    def overlap(self, other: "TTN") -> complex:
        out = np.zeros(2)
        self._check(lib().ttn_overlap(self.h, other.h, _dptr(out)), self.h)
        return complex(out[0], out[1])

    def profile_begin(self, timed: bool = True):
        """Open a profiling window (launches run eagerly and are recorded;
        timed: with HIP events per matvec and per other launch)."""
        f = lib().ttn_profile_begin if timed else lib().ttn_profile_begin_untimed
        self._check(f(self.h), self.h)

    def profile_end(self) -> Profile:
        """Close the window: per-class launch counts, event times, flops."""
        out = Profile()
        self._check(lib().ttn_profile_end(self.h, C.byref(out)), self.h)
        return out

    def profile_launches(self) -> list:
        """The last closed window's contraction launches in launch order."""
        n = lib().ttn_profile_launches(self.h, None, 0)
        self._check(n, self.h)
        arr = (LaunchRec * max(1, n))()
        lib().ttn_profile_launches(self.h, arr, n)
        return [dict(kernel=r.kernel, prec=r.prec, heff=r.heff, splits=r.splits, matvec=r.matvec, flops=r.flops,
                     ms=r.ms) for r in arr[:n]]

    def set_graphs(self, enabled: bool):
        """Replay the step body as a HIP graph (default) or launch eagerly."""
        self._check(lib().ttn_set_graphs(self.h, int(bool(enabled))), self.h)

    def record(self, n_steps: int, ckpt_every: int = 10):
        """Start recording the next n_steps steps for backward()."""
        import torch
        cfg = make_config(self.w, self._keep)
        nbytes = C.c_size_t(0)
        self._check(lib().ttn_adjoint_query(C.byref(cfg), int(n_steps), int(ckpt_every), C.byref(nbytes)), None)
        self.adj_buffer = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        rc = lib().ttn_record_begin(self.h, int(n_steps), int(ckpt_every), C.c_void_p(self.adj_buffer.data_ptr()),
                                    nbytes)
        self._check(rc, self.h)
        return int(nbytes.value)

    def backward(self, target_sites=None, dF: float = 1.0):
        """dF * (dF/dOmega, dF/dDelta), each [N][n_seg], through the recorded steps."""
        ts = np.ascontiguousarray(self.w.target_sites if target_sites is None else target_sites, dtype=np.int32)
        ns = int(np.asarray(self._pulses[1]).shape[1])
        go = np.zeros((self.w.n_sites, ns))
        gd = np.zeros((self.w.n_sites, ns))
        rc = lib().ttn_backward(self.h, len(ts), _iptr(ts), float(dF), _dptr(go), _dptr(gd))
        self._check(rc, self.h)
        return go, gd

    def sample(self, n_shots: int, seed: int, shot0: int = 0, batch: int = 8192):
        """n_shots projective measurements of all sites: (configs [n][N] uint8,
        amplitudes psi(s) [n] complex)."""
        import torch
        nbytes = C.c_size_t(0)
        self._check(lib().ttn_sample_query(self.h, int(max(1, min(batch, n_shots))), C.byref(nbytes)), self.h)
        buf = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        cfg = np.zeros((n_shots, self.w.n_sites), dtype=np.uint8)
        amp = np.zeros(2 * n_shots)
        rc = lib().ttn_sample(self.h, int(n_shots), C.c_uint64(seed), int(shot0), C.c_void_p(buf.data_ptr()), nbytes,
                              cfg.ctypes.data_as(C.POINTER(C.c_uint8)), _dptr(amp))
        self._check(rc, self.h)
        return cfg, amp.view(np.complex128)

    def export_state(self) -> np.ndarray:
        n = lib().ttn_export_state(self.h, None, 0)
        buf = np.zeros(2 * n)
        self._check(lib().ttn_export_state(self.h, _dptr(buf), n), self.h)
        return buf.view(np.complex128)

    def close(self):
        if getattr(self, "h", None):
            lib().ttn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_FIDELITY_FN = None


def _fidelity_function():
    global _FIDELITY_FN
    if _FIDELITY_FN is not None:
        return _FIDELITY_FN
    import torch

    class TTNFidelity(torch.autograd.Function):
        """F = |<GHZ_S|psi_n>|^2 after n TDVP steps of a workload whose pulse
        table is given as tensors, differentiable with respect to that table
        through the library's adjoint (ttn_record_begin + ttn_backward).

        forward(omega, delta, w, n_steps=None, ckpt_every=10, target_sites=None):
        omega, delta are [N][n_seg] float64 tensors (any device; copied to the
        host for ttn_set_pulses); returns F as a 0-d float64 tensor on omega's
        device.  backward returns dF * dF/dOmega and dF * dF/dDelta."""

        @staticmethod
        def forward(ctx, omega, delta, w, n_steps=None, ckpt_every=10, target_sites=None):
            om = omega.detach().to("cpu", torch.float64).numpy()
            de = delta.detach().to("cpu", torch.float64).numpy()
            n = w.n_steps if n_steps is None else int(n_steps)
            g = TTN(w.copy(omega=om, delta=de))
            g.record(n, ckpt_every)
            g.step(n)
            F, _ = g.fidelity(target_sites)
            ctx.g = g
            ctx.target = target_sites
            ctx.dev = omega.device
            return torch.tensor(F, dtype=torch.float64, device=omega.device)

        @staticmethod
        def backward(ctx, gF):
            go, gd = ctx.g.backward(ctx.target, float(gF))
            ctx.g.close()
            ctx.g = None
            return (torch.as_tensor(go, device=ctx.dev), torch.as_tensor(gd, device=ctx.dev), None, None, None,
                    None)

    _FIDELITY_FN = TTNFidelity
    return TTNFidelity


def ttn_fidelity(omega, delta, w, n_steps=None, ckpt_every=10, target_sites=None):
    """Differentiable GHZ fidelity of workload w under the pulse tensors
    (omega, delta): see TTNFidelity."""
    return _fidelity_function().apply(omega, delta, w, n_steps, ckpt_every, target_sites)
