#!/usr/bin/env python3
"""Benchmark: single-site TDVP steps/s of the 8x8, d=4, chi=128 Rydberg TTN
(mixed precision: complex FP32 contractions, FP64 Krylov/QR) on one MI355X,
with the H_eff contraction kernel's achieved TFLOP/s against the FP32 MFMA
peak, the plain FP64 GPU path timed beside it, and the CPU oracle timed on a
bounded sample.  Prints one JSON line.

A step is one full TDVP step (S(dt/2) then S*(dt/2) over all 63 nodes and 62
bonds, environment refresh and program events) of the GHZ-preparation
program; inputs are synthetic and seeded and already resident on the device
when the timed region starts.  The timed steps replay the captured step
graph; the contraction-kernel timings come from the same number of steps
right after them, launched eagerly inside a profiling window.

Beside the headline line's fields the JSON carries: fp64_path (the FP64
path over the same steps and its distance to the mixed result),
forward_adjoint (recorded steps and the backward pass of the fidelity
gradient, mixed and FP64), open_system (the same workload with Rydberg
decay), sampling (10^6 projective-measurement shots), bf16x3_variant (the
BF16x3 precision mode over the same workload and its distance to the FP64
path) and cpu_baseline.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TDVP steps/sec + H_eff MFMA util, 8x8 chi=128; mixed vs FP64 at 1e-5 fidel"
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}
HBM_PEAK_GBS = 8000.0
CONTRACT_SRC = os.path.join(ROOT, "paper_2210_03763_amd", "csrc", "contract.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "heff_contract_f32_8x8_d4_chi128_mixed_hbm_traffic.md")


def measured_traffic(workload_name: str):
    """HBM bytes per contraction launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy kernel), or
    None when the summary is absent, was taken on another workload, or the
    contraction kernel source has changed since the counters were taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            kv[k.strip()] = v.strip().strip("`")
    sha = hashlib.sha256(open(CONTRACT_SRC, "rb").read()).hexdigest()
    if kv.get("contract_source_sha256") != sha or kv.get("workload") != workload_name:
        return None
    try:
        return float(kv["hbm_bytes_per_heff_launch"])
    except (KeyError, ValueError):
        return None


def heff_flops_per_step(w) -> float:
    """Algorithmic real flops of all H_eff and K_eff matvecs of one step:
    24 matvecs (two sweeps x Krylov dimension 12) per node and per bond, each
    chi_L chi_R chi_P [chi_L (1 + s_L) + chi_R (1 + s_L + s_R) + chi_P (1 + s_L
    + s_R)] complex multiply-adds at 8 real flops (parent-leg terms, and the
    right-leg n_j products that only feed them, absent at the root)."""
    N, d, chi = w.n_sites, w.d, w.chi
    K = int(round(math.log2(N)))

    def link(s):
        return 1 if s >= N else min(chi, d ** min(s, 64), d ** min(N - s, 64))

    m = w.krylov_dim
    total = 0.0
    for lvl in range(K):
        nn = N >> (lvl + 1)
        dc = d if lvl == 0 else link(1 << lvl)
        dp = link(1 << (lvl + 1))
        s = 1 << lvl
        root = (lvl == K - 1)
        node = dc * dc * dp * (dc * (1 + s) + dc * (1 + s + (0 if root else s))
                               + (0 if root else dp * (1 + 2 * s)))
        total += nn * 2 * m * node
        if not root:   # bond above each node: (D, 1, D) tensor with 2s sites below
            bond = dp * dp * (dp * (1 + 2 * s) + dp * (1 + 2 * s))
            total += nn * 2 * m * bond
    return 8.0 * total


def host_cpu() -> dict:
    """The host the oracle ran on: logical CPUs of the machine, CPUs this
    process may use, CPU model, and the BLAS/threading torch uses."""
    import torch
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    cfg = torch.__config__.show()
    blas = "MKL" if "BLAS_INFO=mkl" in cfg or "USE_MKL=ON" in cfg else (
        "OpenBLAS" if "openblas" in cfg.lower() else "unknown")
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model,
            "torch_threads": torch.get_num_threads(), "blas": blas}


def cpu_baseline(w, flops_per_step, budget_s=30.0):
    """The oracle (plain CPU FP64) timed on a bounded sample of the same
    workload: environments of the first step are built (untimed), then the
    oracle's H_eff matvec of the largest node is applied repeatedly for about
    `budget_s` seconds.  steps/s = oracle matvec flop rate / H_eff flops per
    step (an upper bound: the oracle's environment and QR work is left out)."""
    import torch
    from oracle import ttn_oracle as O
    threads = torch.get_num_threads()
    st = O.build(w)
    st.set_time(torch.as_tensor(w.seg_edges), torch.as_tensor(w.omega), torch.as_tensor(w.delta),
                0.5 * w.dt)
    st.rebuild_up()
    tr = st.tree
    v = tr.children[tr.root][0]
    st.build_down(v)
    H = st.heff(v)
    DL, DR, DP = tr.dims[v]
    s = len(tr.child_sites(v, 0))
    fl = 8.0 * DL * DR * DP * (DL * (1 + s) + DR * (1 + 2 * s) + DP * (1 + 2 * s))
    x = st.T[v].clone()
    n_done, t0 = 0, time.perf_counter()
    while True:
        x = H(x)
        x = x / torch.linalg.vector_norm(x)
        n_done += 1
        el = time.perf_counter() - t0
        if el > budget_s or n_done >= 64:
            break
    rate = n_done * fl / el
    return {"value": rate / flops_per_step, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "host": host_cpu(),
            "sample": f"{n_done} oracle H_eff matvecs of the level-{tr.level[v]} node "
                      f"({DL}x{DR}x{DP}, {fl / 1e9:.0f} GFLOP each) in {el:.1f} s on CPU "
                      f"({rate / 1e9:.1f} GFLOP/s), scaled by {flops_per_step / 1e12:.1f} TFLOP of "
                      f"H_eff/K_eff matvecs per step; environment/QR work not counted"}


def calibration_copy(mib):
    """A streaming kernel of known traffic (reads and writes mib MiB once),
    run just before the profiled steps so that hardware-counter passes can
    scale their byte counts and tell those dispatches apart."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(f"[bench] calibration copy: {n * 4} bytes read, {n * 4} bytes written", file=sys.stderr,
          flush=True)


def run_gpu(w, steps, warmup, profile=True, calib_mib=0, graphs=True, launch_log=None, timed_window=True):
    """Warm-up steps (the first captures the step graph), `steps` timed steps
    replayed from the graph, then -- with profile -- `steps` more steps in a
    profiling window (launched eagerly, each contraction bracketed by HIP
    events on the handle's stream; launch_log receives the window's launch
    records as JSON)."""
    import torch
    from paper_2210_03763_amd import ttn
    g = ttn.TTN(w, device="cuda:0")
    if not graphs:
        g.set_graphs(False)
    if warmup:
        g.step(warmup)
    torch.cuda.synchronize()
    print(f"[bench] {warmup} warm-up step(s) done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"[bench] {steps} timed step(s) done", file=sys.stderr, flush=True)
    prof = ttn.Profile()
    ms_prof = None
    if profile:
        if calib_mib > 0:
            calibration_copy(calib_mib)
        g.profile_begin(timed=timed_window)
        t2 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        prof = g.profile_end()
        ms_prof = (t3 - t2) * 1e3 / steps
        if launch_log:
            with open(launch_log, "w") as f:
                json.dump({"workload": w.name, "steps": steps, "timed": timed_window,
                           "heff_event_ms": prof.heff.ms, "heff_flops": prof.heff.flops,
                           "launches": g.profile_launches()}, f)
        print(f"[bench] {steps} profiled step(s) done", file=sys.stderr, flush=True)
    F, _ = g.fidelity()
    n2, E = g.observables()
    return g, (t1 - t0) * 1e3 / steps, prof, ms_prof, F, n2, E


def adjoint_target(w):
    """Target sites of the forward+adjoint measurement: the atoms the program
    has rotated at its first step.  Early in the program the all-atom GHZ
    fidelity depends only on the |0...0> amplitude, which no drive touches,
    so its gradient vanishes up to rounding; the GHZ state of the rotated
    atoms has a gradient of order 1e-5 there."""
    return sorted({s for (k, s, _) in w.events if k == 0}) or list(range(w.n_sites))


def run_adjoint(w, steps, ckpt=10, target=None):
    """Forward + adjoint: `steps` recorded steps (a state checkpoint every
    `ckpt` steps) and the backward pass of the GHZ fidelity gradient, timed
    separately.  Returns the timings and the gradient (omega, delta)."""
    import numpy as np
    import torch
    from paper_2210_03763_amd import ttn
    g = ttn.TTN(w, device="cuda:0")
    g.step(1)
    nbytes = g.record(steps, ckpt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    go, gd = g.backward(target_sites=target)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g.close()
    del g
    torch.cuda.empty_cache()
    fwd, bwd = (t1 - t0) / steps, (t2 - t1) / steps
    return {"steps": steps, "ckpt_every": ckpt, "fwd_ms_per_step": round(1e3 * fwd, 2), "bwd_ms_per_step": round(1e3 * bwd, 2),
            "fwd_adj_steps_per_s": round(1.0 / (fwd + bwd), 4), "adjoint_buffer_gib": round(nbytes / 2 ** 30, 2),
            "max_abs_grad": float(max(abs(go).max(), abs(gd).max()))}, np.concatenate([go.ravel(), gd.ravel()])


def run_contract_stage(stage, reps=5, chi=128, precision=1):
    """One H_eff stage of a 128^3 node as a single contraction launch through
    ttn_leg_contract (complex FP32), for kernel-level profiling: A = the left
    block and 16 left-site operators on a shared tensor, B = 16 right-site
    operators, C = the right-leg sum over 17 operator/tensor pairs, D = the
    parent-leg sum over 33 pairs."""
    import torch
    from paper_2210_03763_amd import ttn
    L = ttn.lib()
    L.ttn_leg_contract.restype = C.c_int
    L.ttn_leg_contract.argtypes = [C.c_int32] * 6 + [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                                     C.c_int32, C.c_void_p]
    leg, K, xpo, sm = {"A": (0, 17, 0, 0), "B": (1, 16, 0, 0), "C": (1, 17, 1, 1), "D": (2, 33, 1, 1)}[stage]
    n = chi ** 3
    g = torch.Generator(device="cuda").manual_seed(7)
    ops = torch.randn(K, 2 * chi * chi, dtype=torch.float32, device="cuda", generator=g)
    x = torch.randn(K if xpo else 1, 2 * n, dtype=torch.float32, device="cuda", generator=g)
    y = torch.zeros(1 if sm else K, 2 * n, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rc = L.ttn_leg_contract(precision, leg, chi, chi, chi, K, ops.data_ptr(), x.data_ptr(), xpo, y.data_ptr(),
                                sm, 0, st)
        e1.record()
        torch.cuda.synchronize()
        assert rc == 0
        times.append(e0.elapsed_time(e1))
    ms = min(times[1:]) if reps > 1 else times[0]
    fl = 8.0 * n * chi * K
    return {"contract_stage": stage, "precision": {1: "fp32", 2: "bf16x3"}[precision],
            "shape": f"{chi}^3, {K} operators, leg {leg}", "ms": round(ms, 4),
            "tflops_algorithmic": round(fl / ms / 1e9, 2), "reps": reps}


def run_c5(steps):
    """The 8x8, d = 4, chi = 256 repetition-code program: mixed and FP64
    forward steps/s (one warm-up step each), their distance, and forward +
    adjoint over `steps` recorded steps (checkpoint every 2) with the mixed
    gradient's distance to the FP64 one."""
    import numpy as np
    import torch
    from paper_2210_03763_amd import ttn, workload as W
    w = W.config("c5")
    out = {"workload": w.name, "steps": steps}
    fw = {}
    for prec, key in ((ttn.PREC_FP32, "mixed"), (ttn.PREC_FP64, "fp64"), (ttn.PREC_BF16X3, "bf16x3")):
        g = ttn.TTN(w.copy(precision=prec), device="cuda:0")
        g.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        F, _ = g.fidelity()
        fw[key] = g
        out[f"{key}_ms_per_step"] = round(ms, 1)
        out[f"{key}_F"] = F
        print(f"[bench] c5 {key}: {ms:.0f} ms/step", file=sys.stderr, flush=True)
    ov = fw["mixed"].overlap(fw["fp64"])
    out["abs_dF"] = abs(out["mixed_F"] - out["fp64_F"])
    out["state_infidelity_C"] = 1 - abs(ov) ** 2
    out["mixed_speedup"] = round(out["fp64_ms_per_step"] / out["mixed_ms_per_step"], 3)
    ovb = fw["bf16x3"].overlap(fw["fp64"])
    out["bf16x3_abs_dF"] = abs(out["bf16x3_F"] - out["fp64_F"])
    out["bf16x3_state_infidelity_C"] = 1 - abs(ovb) ** 2
    out["bf16x3_speedup"] = round(out["fp64_ms_per_step"] / out["bf16x3_ms_per_step"], 3)
    for g in fw.values():
        g.close()
    del fw
    torch.cuda.empty_cache()
    grads = {}
    for prec, key in ((ttn.PREC_FP32, "mixed"), (ttn.PREC_FP64, "fp64"), (ttn.PREC_BF16X3, "bf16x3")):
        g = ttn.TTN(w.copy(precision=prec), device="cuda:0")
        g.step(1)
        nbytes = g.record(steps, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        go, gd = g.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        grads[key] = (go, gd)
        out[f"{key}_fwd_adj_ms_per_step"] = round((t2 - t0) * 1e3 / steps, 1)
        out[f"{key}_bwd_ms_per_step"] = round((t2 - t1) * 1e3 / steps, 1)
        out[f"{key}_adjoint_buffer_gib"] = round(nbytes / 2 ** 30, 2)
        print(f"[bench] c5 {key} forward+adjoint done", file=sys.stderr, flush=True)
        g.close()
        del g
        torch.cuda.empty_cache()
    scale = max(np.abs(grads["fp64"][0]).max(), np.abs(grads["fp64"][1]).max())
    out["max_abs_grad_fp64"] = scale
    for key in ("mixed", "bf16x3"):
        err = max(np.abs(grads[key][0] - grads["fp64"][0]).max(), np.abs(grads[key][1] - grads["fp64"][1]).max())
        out[f"{key}_max_abs_grad_diff"] = err
        out[f"{key}_speedup_fwd_adj"] = round(out["fp64_fwd_adj_ms_per_step"] / out[f"{key}_fwd_adj_ms_per_step"], 3)
    return out


def run_bf16(w, steps, warmup, graphs=True):
    """The BF16x3 precision mode on the same workload: timed steps and its
    distance to the FP64 path after the same number of steps."""
    import torch
    from paper_2210_03763_amd import ttn
    gb, ms, _, _, Fb, n2b, _ = run_gpu(w.copy(precision=ttn.PREC_BF16X3), steps, warmup, profile=False,
                                       graphs=graphs)
    g64 = ttn.TTN(w.copy(precision=ttn.PREC_FP64), device="cuda:0")
    g64.step(warmup + steps)
    F64, _ = g64.fidelity()
    ov = gb.overlap(g64)
    out = {"ms_per_step": round(ms, 3), "steps_per_s": round(1e3 / ms, 4), "after_steps": warmup + steps,
           "abs_dF_vs_fp64": abs(Fb - F64), "state_infidelity_C_vs_fp64": 1 - abs(ov) ** 2}
    gb.close()
    g64.close()
    torch.cuda.empty_cache()
    return out


def run_two_site(steps, chi=12):
    """Two-site (two-tensor) TDVP, FP64, on the 8x8, d = 3 GHZ-preparation
    program at bond dimension chi (12 is the paper's): one warm-up step (it
    captures the step graph), `steps` timed steps, then one step in a
    profiling window for the contraction launches (the two-site matvecs are
    FP64) and the largest discarded weight of the timed steps."""
    import torch
    from paper_2210_03763_amd import ttn, workload as W
    w = W.make_ghz_program(8, 8, 3, chi, 200, 0.005, 2210037632, eps=0.05,
                           name=f"8x8 d3 chi{chi} GHZ program, two-site").copy(update=ttn.UPDATE_TWO_SITE)
    g = ttn.TTN(w, device="cuda:0")
    g.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = g.step(steps, stats=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    g.profile_begin()
    g.step(1)
    p = g.profile_end()
    F, _ = g.fidelity()
    g.close()
    k = p.heff
    ach = (k.flops / 1e12) / (k.ms / 1e3) if k.ms > 0 else 0.0
    return {"workload": w.name, "steps": steps, "ms_per_step": round(ms, 2), "steps_per_s": round(1e3 / ms, 3),
            "max_discarded_weight": max(s["max_discarded"] for s in stats), "fidelity": F,
            "matvec_launches": int(k.launches), "matvec_tflops_fp64": round(ach, 3),
            "matvec_frac_of_fp64_peak": round(ach / PEAK_TFLOPS["fp64"], 4),
            "matvec_ms_per_step": round(k.ms, 2), "note": "ms_per_step includes the statistics read-back per step"}


def run_c4_gradient(n_params=16, h=1e-6, seed=2210037634, part=(0, 1)):
    """The 8x8, d = 3, chi = 64 gradient workload at its stated size: 200
    recorded steps with a checkpoint every 10, the gradient of the all-atom
    GHZ fidelity with respect to the 64 x 8 x {Omega, Delta} pulse table by
    the adjoint (FP64), and central differences of the device forward map at
    n_params parameters drawn with numpy PCG64(seed) (step h)."""
    import numpy as np
    import torch
    from paper_2210_03763_amd import ttn, workload as W
    w = W.config("c4")
    n = w.n_steps
    os.environ["TTN_PROGRESS"] = "1"      # the backward pass reports its checkpoint blocks
    g = ttn.TTN(w, device="cuda:0")
    nbytes = g.record(n, w.ckpt_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for done in range(0, n, 20):
        g.step(min(20, n - done))
        print(f"[bench] c4 recorded steps: {min(n, done + 20)} of {n}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    F, _ = g.fidelity()
    print(f"[bench] c4 forward: {t1 - t0:.1f} s", file=sys.stderr, flush=True)
    go, gd = g.backward()
    del os.environ["TTN_PROGRESS"]
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g.close()
    del g
    torch.cuda.empty_cache()
    grad = np.concatenate([go.ravel(), gd.ravel()])
    scale = float(np.abs(grad).max())
    rng = np.random.Generator(np.random.PCG64(seed))
    picks = sorted(rng.choice(grad.size, size=n_params, replace=False).tolist())
    picks = picks[part[0]::part[1]]     # this call's share of the sampled parameters
    rows = []
    t3 = time.perf_counter()
    for idx in picks:
        arr = w.omega if idx < go.size else w.delta
        i, sg = divmod(idx % go.size, go.shape[1])
        base = arr[i, sg]
        Fs = []
        for x in (base + h, base - h):
            arr[i, sg] = x
            gg = ttn.TTN(w, device="cuda:0")
            gg.step(n)
            Fs.append(gg.fidelity()[0])
            gg.close()
        arr[i, sg] = base
        fd = (Fs[0] - Fs[1]) / (2 * h)
        rows.append({"param": ("omega" if idx < go.size else "delta") + f"[{i},{sg}]", "adjoint": float(grad[idx]),
                     "central_difference": fd})
        print(f"[bench] c4 {rows[-1]} ({time.perf_counter() - t3:.0f} s)", file=sys.stderr, flush=True)
    t4 = time.perf_counter()
    diffs = [abs(r["adjoint"] - r["central_difference"]) for r in rows]
    return {"workload": w.name, "recorded_steps": n, "ckpt_every": w.ckpt_every, "F": F, "max_abs_grad": scale,
            "fd_step": h, "fd_params": rows, "max_abs_diff": max(diffs),
            "max_rel_diff_to_max_grad": max(diffs) / scale if scale > 0 else None,
            "fwd_s": round(t1 - t0, 2), "bwd_s": round(t2 - t1, 2), "fd_s": round(t4 - t3, 1),
            "adjoint_buffer_gib": round(nbytes / 2 ** 30, 2)}


def run_open(w, steps, warmup, gamma):
    """Open-system mode (Eq. (eq:hoqs): -i gamma |r><r| per site, Arnoldi
    local exponentials) on the same workload: timed steps from the step
    graph, then the no-decay probability ||psi||^2, the remaining Rydberg
    population P_R = sum_i <psi|n_i|psi> and the GHZ fidelity of the
    unnormalised state (lost norm counts as fidelity zero)."""
    import torch
    from paper_2210_03763_amd import ttn
    g = ttn.TTN(w.copy(gamma=gamma), device="cuda:0")
    if warmup:
        g.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    n2, _ = g.observables()
    pop = g.rydberg_population()
    F, _ = g.fidelity()
    g.close()
    del g
    torch.cuda.empty_cache()
    return {"gamma": gamma, "steps": steps, "ms_per_step": round(ms, 3), "steps_per_s": round(1e3 / ms, 4),
            "after_steps": warmup + steps, "norm2": n2, "rydberg_population_P_R": pop, "fidelity": F}


def sample_flops_per_shot(w) -> float:
    """Algorithmic real flops of one shot: at every node above the bottom the
    batch GEMMs B = Q u and phi = Q^T (phi_L (x) phi_R), 8 D_L D_R D_P each."""
    N, d, chi = w.n_sites, w.d, w.chi
    K = int(round(math.log2(N)))

    def link(s):
        return 1 if s >= N else min(chi, d ** min(s, 64), d ** min(N - s, 64))

    total = 0.0
    for lvl in range(1, K):
        nn = N >> (lvl + 1)
        dc, dp = link(1 << lvl), link(1 << (lvl + 1))
        total += nn * 2 * 8.0 * dc * dc * dp
    return total


def run_sampling(w, shots, warm_steps=2):
    import torch
    from paper_2210_03763_amd import ttn
    g = ttn.TTN(w.copy(precision=ttn.PREC_FP64), device="cuda:0")
    g.step(warm_steps)
    g.sample(1000, 1)           # first-use costs outside the timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cfg, amp = g.sample(shots, 2210037635)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    g.close()
    fl = sample_flops_per_shot(w) * shots
    import numpy as np
    _, first = np.unique(cfg, axis=0, return_index=True)
    return {"shots": shots, "seconds": round(el, 3), "shots_per_s": round(shots / el, 1),
            "gemm_tflop": round(fl / 1e12, 2), "gemm_tflops_over_the_call": round(fl / el / 1e12, 2),
            "fp64_mfma_peak": PEAK_TFLOPS["fp64"], "state": f"FP64 network after {warm_steps} steps",
            "distinct_configs": int(len(first)),
            "probability_covered": float((abs(amp[first]) ** 2).sum())}


# ---------------------------------------------------------------------------
# rocprofv3 summaries (python bench.py --summarize-profile DIR)
# ---------------------------------------------------------------------------
# DIR holds up to three rocprofv3 output folders of bench.py runs with
# --calib-copy-mib and --launch-log: trace/ (--kernel-trace --stats), fetch/
# (--pmc FETCH_SIZE) and write/ (--pmc WRITE_SIZE), each with its
# launches.json.  A run's profiling window starts right after the calibration
# kernel (the dispatch whose name contains "neg_kernel"); in it, contraction
# launches are the dispatches named k_cgemm_mfma<...>, k_cgemm_bf16x3<...> or
# k_cgemm<...> (the main kernels), each followed by its k_splitk_reduce* dispatch
# when the launch record says split-K > 1.  The i-th main dispatch after the
# calibration kernel is the i-th record of launches.json; its kernel class and
# operand precision are checked against the kernel name.

CONTRACT_MAIN = ("k_cgemm_mfma<", "k_cgemm_bf16x3<", "k_cgemm<")
KERNEL_CLASS = {"k_cgemm<": 1, "k_cgemm_mfma<": 2, "k_cgemm_bf16x3<": 3}


def _short(name: str) -> str:
    """Kernel name without namespace, return type and argument list."""
    n = name
    for pre in ("void ", "ttn::(anonymous namespace)::", "(anonymous namespace)::"):
        n = n.replace(pre, "")
    depth, cut = 0, None
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    return n[:cut] if cut else n


def _main_class(short: str):
    for pre in CONTRACT_MAIN:
        if short.startswith(pre):
            return KERNEL_CLASS[pre], ("double" if short[len(pre):].startswith("double") else "float")
    return None, None


def _read_rows(folder: str, suffix: str):
    import csv
    import glob
    import gzip
    hits = sorted(glob.glob(os.path.join(folder, "**", f"*{suffix}"), recursive=True) +
                  glob.glob(os.path.join(folder, "**", f"*{suffix}.gz"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {folder}")
    path = hits[0]
    f = gzip.open(path, "rt") if path.endswith(".gz") else open(path)
    with f:
        return list(csv.DictReader(f)), path


def match_window(dispatches, launches):
    """dispatches: [(dispatch_id, kernel_name, payload)] in dispatch order.
    Returns (first, last, pairs): the window's dispatch index range and, per
    launch record, (record, main index, reduction index or None)."""
    cal = [i for i, d in enumerate(dispatches) if "neg_kernel" in d[1]]
    if not cal:
        raise ValueError("calibration kernel not found")
    i = cal[-1] + 1
    pairs = []
    for rec in launches:
        while i < len(dispatches) and _main_class(_short(dispatches[i][1]))[0] is None:
            i += 1
        if i >= len(dispatches):
            raise ValueError(f"ran out of dispatches at launch {len(pairs)}")
        cls, prec = _main_class(_short(dispatches[i][1]))
        want_prec = "float" if rec["prec"] == 1 else "double"
        if cls != rec["kernel"] or prec != want_prec:
            raise ValueError(f"launch {len(pairs)}: dispatch {_short(dispatches[i][1])} does not match "
                             f"record class {rec['kernel']} / {want_prec}")
        main = i
        i += 1
        red = None
        if rec["splits"] > 1:
            while i < len(dispatches) and "k_splitk_reduce" not in dispatches[i][1]:
                if _main_class(_short(dispatches[i][1]))[0] is not None:
                    raise ValueError(f"launch {len(pairs)}: split-K reduction missing")
                i += 1
            red = i
            i += 1
        pairs.append((rec, main, red))
    return cal[-1] + 1, i - 1, pairs


def _trace_summary(folder, launches_json):
    rows, path = _read_rows(folder, "kernel_trace.csv")
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    disp = [(int(r["Dispatch_Id"]), r["Kernel_Name"],
             (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6) for r in rows]
    L = json.load(open(launches_json))
    first, last, pairs = match_window(disp, L["launches"])
    dur = lambda k: disp[k][2] if k is not None else 0.0  # noqa: E731

    def cls(sel):
        ps = [p for p in pairs if sel(p[0])]
        ms = sum(dur(m) + dur(r) for _, m, r in ps)
        fl = sum(p[0]["flops"] for p in ps)
        ev = sum(p[0]["ms"] for p in ps)
        return {"launches": len(ps), "ms": ms, "avg_ms": ms / max(1, len(ps)), "flops": fl,
                "tflops": fl / 1e12 / (ms / 1e3) if ms > 0 else 0.0, "event_ms": ev,
                "reductions": sum(1 for _, _, r in ps if r is not None)}
    # the launches of each H_eff / K_eff matvec, spanned from its first main
    # kernel's start to its last kernel's end
    mv = {}
    for rec, m, r in pairs:
        if rec["heff"] == 1 and rec["prec"] == 1:
            a, b = mv.get(rec["matvec"], (None, None))
            last = r if r is not None else m
            mv[rec["matvec"]] = (m if a is None else a, last)
    span_heff = sum((int(rows[b]["End_Timestamp"]) - int(rows[a]["Start_Timestamp"])) * 1e-6 for a, b in mv.values())
    fam = {}
    for k in range(first, last + 1):
        n = _short(disp[k][1])
        c, t = fam.get(n, (0, 0.0))
        fam[n] = (c + 1, t + disp[k][2])
    span = (int(rows[last]["End_Timestamp"]) - int(rows[first]["Start_Timestamp"])) * 1e-6
    return dict(path=path, workload=L["workload"], steps=L["steps"], first=first, last=last, n_matvecs=len(mv),
                heff_span_ms=span_heff, heff_event_ms=L.get("heff_event_ms"),
                heff=cls(lambda r: r["heff"] == 1 and r["prec"] == 1),
                f32=cls(lambda r: r["prec"] == 1), f64=cls(lambda r: r["prec"] == 0),
                families=fam, kernel_ms=sum(v[1] for v in fam.values()), span_ms=span)


def _counter_summary(folder, launches_json, counter):
    rows, path = _read_rows(folder, "counter_collection.csv")
    by = {}
    for r in rows:
        if r.get("Counter_Name", counter) != counter:
            continue
        d = int(r["Dispatch_Id"])
        nm, v = by.get(d, (r["Kernel_Name"], 0.0))
        by[d] = (nm, v + float(r["Counter_Value"]))
    disp = [(d, by[d][0], by[d][1]) for d in sorted(by)]
    L = json.load(open(launches_json))
    first, last, pairs = match_window(disp, L["launches"])
    cal = disp[first - 1][2]
    val = lambda k: disp[k][2] if k is not None else 0.0  # noqa: E731
    heff = [p for p in pairs if p[0]["heff"] == 1 and p[0]["prec"] == 1]
    allf = [p for p in pairs if p[0]["prec"] == 1]
    return dict(path=path, calib_kib=cal, launches=len(pairs),
                heff_kib=sum(val(m) + val(r) for _, m, r in heff), n_heff=len(heff),
                f32_kib=sum(val(m) + val(r) for _, m, r in allf), n_f32=len(allf))


def summarize_profile(profdir, calib_mib=256, out_dir=None):
    """Writes the kernel-trace and HBM-traffic summaries under profiles/."""
    import hashlib
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    written = []
    base = ("--steps 1 --warmup 1 --no-fp64 --no-cpu --adjoint-steps 0 --sample-shots 0 --open-gamma 0 "
            "--bf16-steps 0 --two-site-steps 0 --calib-copy-mib 256")
    tdir = os.path.join(profdir, "trace")
    if os.path.isdir(tdir):
        t = _trace_summary(tdir, os.path.join(tdir, "launches.json"))
        h, f = t["heff"], t["f32"]
        lines = [
            "# Kernel trace: one mixed-precision TDVP step, 8x8, d=4, chi=128",
            "",
            f"Workload: {t['workload']} (the bench workload: GHZ-preparation program, Krylov dimension 12).",
            "Window: the dispatches of the profiled step (launched eagerly inside the library's profiling",
            "window), from the one after the calibration kernel (name containing `neg_kernel`) to the",
            "window's last contraction launch.",
            "",
            "Command (R = repository root on the GPU box), then the summary:",
            "",
            "```",
            f"cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv "
            f"-d $R/gpurun_out/prof/trace -o run -- python3 $R/bench.py {base} "
            f"--launch-log $R/gpurun_out/prof/trace/launches.json",
            "python bench.py --summarize-profile gpurun_out/prof",
            "```",
            "",
            "Kernel-name filter of the contraction launches: main kernels `k_cgemm_mfma<...>`,",
            "`k_cgemm_bf16x3<...>`, `k_cgemm<...>`; each followed by its `k_splitk_reduce<...>` or",
            "`k_splitk_reduce_vec<...>` dispatch when the launch record has split-K > 1 (both counted).",
            "The i-th main dispatch is the i-th record of the library's launch log (kernel class and",
            "operand precision checked); H_eff/K_eff launches are the records flagged heff.",
            "",
            f"Kernel time in the window: {t['kernel_ms']:.1f} ms over {t['last'] - t['first'] + 1} dispatches; "
            f"first-to-last dispatch span {t['span_ms']:.1f} ms.",
            "",
            "| launch class | launches | with reduction | device ms (main + reduction) | avg ms per launch | "
            "algorithmic TFLOP/s |",
            "|---|---|---|---|---|---|",
        ]
        for key, lab in (("heff", "H_eff/K_eff matvecs, FP32 (roofline kernel)"), ("f32", "all FP32 contractions"),
                         ("f64", "all FP64 contractions (gauge moves)")):
            c = t[key]
            lines.append(f"| {lab} | {c['launches']} | {c['reductions']} | {c['ms']:.2f} | {c['avg_ms']:.5f} | "
                         f"{c['tflops']:.1f} |")
        ev = t["heff_event_ms"] or 0.0
        lines += ["",
                  "H_eff/K_eff launches, three measures of the same work (the library times each matvec's",
                  "launches between one event pair; `roofline.avg_launch_ms` of bench.py is that event time per",
                  "launch):", "",
                  f"- heff_launches: {h['launches']}",
                  f"- heff_kernel_ms (sum of kernel durations, main + reduction): {h['ms']:.2f}",
                  f"- heff_span_ms (first kernel start to last kernel end of each matvec, {t['n_matvecs']} matvecs): "
                  f"{t['heff_span_ms']:.2f}",
                  f"- heff_event_ms (library events, this run): {ev:.2f}",
                  f"- heff_avg_launch_ms: {h['avg_ms']:.5f} (kernels), {t['heff_span_ms'] / h['launches']:.5f} "
                  f"(spans), {ev / h['launches']:.5f} (events)",
                  f"- heff_tflops_algorithmic: {h['tflops']:.2f} (kernels), "
                  f"{h['flops'] / 1e12 / (t['heff_span_ms'] / 1e3):.2f} (spans)",
                  f"- heff_frac_of_fp32_peak: {h['tflops'] / PEAK_TFLOPS['fp32']:.4f} (kernels), "
                  f"{h['flops'] / 1e12 / (t['heff_span_ms'] / 1e3) / PEAK_TFLOPS['fp32']:.4f} (spans)", "",
                  "| kernel | calls | total ms | avg us | % of window |", "|---|---|---|---|---|"]
        for n, (c, ms) in sorted(t["families"].items(), key=lambda kv: -kv[1][1])[:40]:
            lines.append(f"| `{n}` | {c} | {ms:.2f} | {1e3 * ms / c:.1f} | {100 * ms / t['kernel_ms']:.1f} |")
        p = os.path.join(out_dir, "tdvp_step_8x8_d4_chi128_mixed_kernel_trace.md")
        open(p, "w").write("\n".join(lines) + "\n")
        written.append(p)
    fdir, wdir = os.path.join(profdir, "fetch"), os.path.join(profdir, "write")
    if os.path.isdir(fdir) and os.path.isdir(wdir):
        fs = _counter_summary(fdir, os.path.join(fdir, "launches.json"), "FETCH_SIZE")
        ws = _counter_summary(wdir, os.path.join(wdir, "launches.json"), "WRITE_SIZE")
        known = calib_mib * 1024.0
        ff, wf = known / fs["calib_kib"], known / ws["calib_kib"]
        fb = fs["heff_kib"] * 1024 * ff / fs["n_heff"]
        wb = ws["heff_kib"] * 1024 * wf / ws["n_heff"]
        fba = fs["f32_kib"] * 1024 * ff / fs["n_f32"]
        wba = ws["f32_kib"] * 1024 * wf / ws["n_f32"]
        sha = hashlib.sha256(open(CONTRACT_SRC, "rb").read()).hexdigest()
        L = json.load(open(os.path.join(fdir, "launches.json")))
        cmd = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 420 rocprofv3 --pmc {c} --kernel-include-regex "
               "\"k_cgemm|k_splitk_reduce|neg_kernel\" --output-format csv -d $R/gpurun_out/prof/{d} -o run -- "
               "python3 $R/bench.py {b} --no-graphs --untimed-window --launch-log $R/gpurun_out/prof/{d}/launches.json")
        lines = [
            "# HBM traffic of the H_eff/K_eff contraction launches, 8x8, d=4, chi=128 (mixed)",
            "",
            "Two counter passes, one counter each (R = repository root on the GPU box), then the summary:",
            "",
            "```",
            cmd.format(c="FETCH_SIZE", d="fetch", b=base),
            cmd.format(c="WRITE_SIZE", d="write", b=base),
            "python bench.py --summarize-profile gpurun_out/prof",
            "```",
            "",
            "Kernel-name filter: the counter passes record only dispatches matching",
            "`k_cgemm|k_splitk_reduce|neg_kernel`.  Window and launch matching as in the kernel-trace",
            "summary: the i-th main contraction dispatch after the calibration kernel is the i-th record of",
            "the launch log; a launch's bytes are its main kernel's plus its split-K reduction's.  Counter",
            "values (KiB per dispatch) are scaled by known bytes / counter reading of the calibration kernel",
            f"(a streaming kernel that reads and writes {calib_mib} MiB once).",
            "",
            f"- workload: {L['workload']}",
            f"- contract_source_sha256: `{sha}`",
            f"- calibration FETCH_SIZE reading: {fs['calib_kib']:.1f} KiB for {known:.0f} KiB read (factor {ff:.4f})",
            f"- calibration WRITE_SIZE reading: {ws['calib_kib']:.1f} KiB for {known:.0f} KiB written "
            f"(factor {wf:.4f})",
            f"- heff_launches: {fs['n_heff']}",
            f"- fetch_bytes_per_heff_launch: {fb:.0f}",
            f"- write_bytes_per_heff_launch: {wb:.0f}",
            f"- hbm_bytes_per_heff_launch: {fb + wb:.0f}",
            f"- fp32_contraction_launches: {fs['n_f32']}",
            f"- hbm_bytes_per_fp32_launch: {fba + wba:.0f}",
        ]
        p = os.path.join(out_dir, "heff_contract_f32_8x8_d4_chi128_mixed_hbm_traffic.md")
        open(p, "w").write("\n".join(lines) + "\n")
        written.append(p)
    return written


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=25.0)
    ap.add_argument("--adjoint-steps", type=int, default=6,
                    help="recorded steps of the forward+adjoint measurement (0: skip)")
    ap.add_argument("--adjoint-ckpt", type=int, default=1,
                    help="state checkpoint interval of the forward+adjoint measurement")
    ap.add_argument("--sample-shots", type=int, default=1000000,
                    help="projective-measurement shots of the sampling measurement (0: skip)")
    ap.add_argument("--open-gamma", type=float, default=0.02,
                    help="decay rate of the open-system measurement (0: skip)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every step eagerly (for counter collection; kernels are the same)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    ap.add_argument("--untimed-window", action="store_true",
                    help="profiling window without HIP events (for hardware-counter passes)")
    ap.add_argument("--launch-log", default=None,
                    help="write the profiling window's contraction launch records (JSON) here")
    ap.add_argument("--bf16-steps", type=int, default=2,
                    help="also time the BF16x3 precision mode over this many steps")
    ap.add_argument("--c4-fd", type=int, default=0,
                    help="also run the 8x8 d=3 chi=64 gradient at its stated size (200 recorded steps, checkpoint "
                         "every 10) against central differences at this many parameters (0: skip)")
    ap.add_argument("--c4-fd-part", default="0/1", metavar="I/K",
                    help="central differences only at every K-th sampled parameter starting at I")
    ap.add_argument("--two-site-steps", type=int, default=2,
                    help="also time the two-site update on the 8x8 d=3 GHZ program at chi 12 and 16 (0: skip)")
    ap.add_argument("--c5-steps", type=int, default=0,
                    help="also measure the 8x8 d=4 chi=256 repetition-code program over this many steps")
    ap.add_argument("--contract-stage", choices=["A", "B", "C", "D"], default=None,
                    help="time one H_eff contraction stage of a 128^3 node instead (kernel profiling)")
    ap.add_argument("--contract-precision", choices=["fp32", "bf16x3"], default="fp32",
                    help="arithmetic of --contract-stage")
    ap.add_argument("--summarize-profile", default=None, metavar="DIR",
                    help="write the profiles/ summaries from rocprofv3 output under DIR (no GPU needed)")
    args = ap.parse_args()
    if args.summarize_profile:
        for p in summarize_profile(args.summarize_profile, args.calib_copy_mib or 256):
            print(p, flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the TDVP sweep is sequential "
              f"over tree nodes and the library has no multi-GPU path", file=sys.stderr, flush=True)
        sys.exit(2)

    import torch
    from paper_2210_03763_amd import ttn, workload as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.contract_stage:
        print(json.dumps(run_contract_stage(args.contract_stage,
                                            precision=2 if args.contract_precision == "bf16x3" else 1)), flush=True)
        return
    print(f"[bench] building workload {args.config}", file=sys.stderr, flush=True)
    w = W.config(args.config)
    fps = heff_flops_per_step(w)
    print(f"[bench] mixed run: warmup {args.warmup}, timed {args.steps} steps", file=sys.stderr, flush=True)
    gm, ms_mixed, prof, ms_prof, F_m, n2_m, E_m = run_gpu(w, args.steps, args.warmup,
                                                          calib_mib=args.calib_copy_mib,
                                                          graphs=not args.no_graphs,
                                                          launch_log=args.launch_log,
                                                          timed_window=not args.untimed_window)
    print(f"[bench] mixed {ms_mixed:.1f} ms/step F={F_m:.12f}", file=sys.stderr, flush=True)
    dt = "fp32" if w.precision == ttn.PREC_FP32 else "fp64"
    kall = prof.gemm_f32 if w.precision == ttn.PREC_FP32 else prof.gemm_f64
    k = prof.heff          # the H_eff / K_eff matvec launches: the metric's kernel
    avg_ms = k.ms / max(1, k.launches)
    achieved = (k.flops / 1e12) / (k.ms / 1e3) if k.ms > 0 else 0.0
    ach_all = (kall.flops / 1e12) / (kall.ms / 1e3) if kall.ms > 0 else 0.0
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[dt], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_TFLOPS[dt], 4),
            "traffic": measured_traffic(w.name) if dt == "fp32" else None,
            "kernel": f"H_eff/K_eff matvec launches of the complex {dt.upper()} contraction kernel "
                      f"(k_cgemm_mfma / k_cgemm with their split-K reductions); each matvec's launches run "
                      f"back to back between one pair of HIP events",
            "launches": int(k.launches), "avg_launch_ms": round(avg_ms, 5),
            "algorithmic_gflop_per_launch": round(k.flops / max(1, k.launches) / 1e9, 4),
            "matvecs": int(prof.matvecs),
            "all_contractions": {"launches": int(kall.launches), "achieved": round(ach_all, 3),
                                 "frac": round(ach_all / PEAK_TFLOPS[dt], 4),
                                 "avg_launch_ms": round(kall.ms / max(1, kall.launches), 5),
                                 "heff_share_of_flops": round(k.flops / max(1.0, kall.flops), 4)},
            "window": f"the {args.steps} steps after the timed ones, launched eagerly inside a profiling "
                      f"window ({ms_prof:.1f} ms/step there); kernel durations do not depend on graph replay"}
    def vec(p):
        gbs = p.bytes / 1e9 / (p.ms / 1e3) if p.ms > 0 else 0.0
        return {"calls": int(p.calls), "ms_per_step": round(p.ms / args.steps, 3),
                "gbytes_per_step": round(p.bytes / 1e9 / args.steps, 3), "achieved_gb_per_s": round(gbs, 1),
                "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
    hbm = {"peak_gb_per_s": HBM_PEAK_GBS,
           "lanczos_vectors_all": vec(prof.lanczos),
           "lanczos_vectors_ge_2^20": vec(prof.lanczos_large),
           "bytes": "what the Lanczos vector kernels read and write by construction (16 B per complex FP64 "
                    "element, 8 B per FP32 one), HIP events around each call in the profiling window"}
    out = {"metric": METRIC, "value": round(1e3 / ms_mixed, 4), "unit": "steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_mixed, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dt,
           "data": "synthetic (seeded GHZ-preparation pulse program, dressed product state)",
           "config": {"workload": w.name, "lattice": f"{w.Lx}x{w.Ly}", "d": w.d, "chi": w.chi,
                      "krylov_dim": w.krylov_dim, "dt": w.dt, "program_steps": w.n_steps,
                      "precision": "complex FP32 contractions, FP64 Lanczos/QR/environments"
                      if dt == "fp32" else "FP64",
                      "heff_tflop_per_step": round(fps / 1e12, 3)},
           "roofline": roof, "hbm_bound_kernels": hbm}
    if not args.no_fp64 and w.precision == ttn.PREC_FP32:
        w64 = w.copy(precision=ttn.PREC_FP64)
        print(f"[bench] fp64 run: {args.steps} steps", file=sys.stderr, flush=True)
        g64, ms64, _, _, _, _, _ = run_gpu(w64, args.steps, args.warmup, profile=False)
        g64.step(args.steps)                      # same step count as the mixed run
        F64, _ = g64.fidelity()
        n2_64, E64 = g64.observables()
        ov = gm.overlap(g64)
        out["fp64_path"] = {"ms_per_step": round(ms64, 3), "steps_per_s": round(1e3 / ms64, 4),
                            "mixed_speedup": round(ms64 / ms_mixed, 3),
                            "abs_dF": abs(F_m - F64), "state_infidelity_C": 1 - abs(ov) ** 2,
                            "abs_dnorm2": abs(n2_m - n2_64), "abs_dE": abs(E_m - E64),
                            "after_steps": 2 * args.steps + args.warmup}
        g64.close()
    gm.close()
    if args.adjoint_steps > 0:
        import numpy as np
        print(f"[bench] forward+adjoint: {args.adjoint_steps} recorded steps", file=sys.stderr, flush=True)
        tgt = adjoint_target(w)
        adj = {"target_sites": tgt}
        grads = {}
        legs = [("mixed", w.precision)]
        if not args.no_fp64 and w.precision == ttn.PREC_FP32:
            legs += [("fp64", ttn.PREC_FP64)]
            if args.bf16_steps > 0:
                legs += [("bf16x3", ttn.PREC_BF16X3)]
        for key, prec in legs:
            adj[key], grads[key] = run_adjoint(w.copy(precision=prec), args.adjoint_steps, args.adjoint_ckpt, tgt)
        if "fp64" in grads:
            tot = lambda k: adj[k]["fwd_ms_per_step"] + adj[k]["bwd_ms_per_step"]  # noqa: E731
            scale = float(np.abs(grads["fp64"]).max())
            adj["max_abs_grad_fp64"] = scale
            for key in grads:
                if key == "fp64":
                    continue
                e = float(np.abs(grads[key] - grads["fp64"]).max())
                adj[f"{key}_speedup_fwd_adj"] = round(tot("fp64") / max(1e-9, tot(key)), 3)
                adj[f"{key}_max_abs_grad_diff"] = e
                adj[f"{key}_max_rel_grad_diff"] = e / scale if scale > 0 else None
        out["forward_adjoint"] = adj
    if args.open_gamma > 0:
        print(f"[bench] open system: gamma {args.open_gamma}, {args.steps} steps", file=sys.stderr, flush=True)
        out["open_system"] = run_open(w, args.steps, args.warmup, args.open_gamma)
        out["open_system"]["closed_ms_per_step"] = round(ms_mixed, 3)
    if args.bf16_steps > 0:
        print(f"[bench] BF16x3 mode: {args.bf16_steps} steps", file=sys.stderr, flush=True)
        out["bf16x3_variant"] = run_bf16(w, args.bf16_steps, args.warmup, graphs=not args.no_graphs)
    if args.c5_steps > 0:
        print(f"[bench] chi=256 repetition code: {args.c5_steps} steps", file=sys.stderr, flush=True)
        out["chi256_repetition_code"] = run_c5(args.c5_steps)
    if args.c4_fd > 0:
        print(f"[bench] 8x8 chi=64 gradient, 200 recorded steps, {args.c4_fd} central differences",
              file=sys.stderr, flush=True)
        part = tuple(int(x) for x in args.c4_fd_part.split("/"))
        out["c4_gradient"] = run_c4_gradient(args.c4_fd, part=part)
    if args.two_site_steps > 0:
        print(f"[bench] two-site update: {args.two_site_steps} steps", file=sys.stderr, flush=True)
        out["two_site"] = [run_two_site(args.two_site_steps, chi) for chi in (12, 16)]
    if args.sample_shots > 0:
        print(f"[bench] sampling: {args.sample_shots} shots", file=sys.stderr, flush=True)
        out["sampling"] = run_sampling(w, args.sample_shots)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w.copy(precision=0), fps, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
