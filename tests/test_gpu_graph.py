"""The step body replayed as a HIP graph gives the same states as eager
launches: two handles of the same workload, one with graphs disabled, are
stepped one step at a time with eager work (fidelity, observables, a local
expectation) and synchronisations between the replays; every replay's state
must equal the eager state exactly (same kernels on the same data)."""
import numpy as np
import pytest
import torch

from paper_2210_03763_amd import ttn as T
from paper_2210_03763_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["c1-ent", "ghz2x4", "c1-ent-mixed"])
def test_graph_replays_equal_eager_steps(name):
    if name == "ghz2x4":
        w = W.make_ghz_program(4, 2, 3, 6, 8, 0.1, seed=31, n_layers=4, seg_per_layer=2, eps=0.05)
    elif name == "c1-ent-mixed":
        w = W.config("c1-ent").copy(precision=T.PREC_FP32)
    else:
        w = W.config("c1-ent")
    print(f"[graph] {name}", flush=True)
    ga, gb = T.TTN(w), T.TTN(w)
    gb.set_graphs(False)
    n_op = np.diag([0, 0, 1.0]).astype(complex)
    for k in range(5):
        ga.step(1)
        gb.step(1)
        torch.cuda.synchronize()
        fa, fb = ga.fidelity()[0], gb.fidelity()[0]
        ea, eb = ga.observables(), gb.observables()
        la, lb = ga.local_expectation(k, n_op), gb.local_expectation(k, n_op)
        sa, sb = ga.export_state(), gb.export_state()
        assert np.array_equal(sa, sb), (name, k, np.abs(sa - sb).max())
        assert fa == fb and ea == eb and la == lb
    ga.close()
    gb.close()


def test_profile_window_with_graph_replays():
    w = W.config("c1-ent").copy(precision=T.PREC_FP32)
    res = []
    for graphs in (True, False):
        g = T.TTN(w)
        g.set_graphs(graphs)
        g.step(1)
        g.profile_begin()
        g.step(2)
        p = g.profile_end()
        recs = g.profile_launches()
        assert len(recs) == p.gemm_f32.launches + p.gemm_f64.launches
        # matvec launches are timed per matvec (ms -1 each), the rest one by one
        assert all((r["ms"] < 0) == (r["heff"] == 1) for r in recs)
        single = sum(r["ms"] for r in recs if r["ms"] >= 0)
        assert abs(single + p.heff.ms - (p.gemm_f32.ms + p.gemm_f64.ms)) < 1e-6 * max(1.0, p.gemm_f32.ms)
        res.append(p)
        g.close()
    a, b = res
    print(f"[graph] launches {a.gemm_f32.launches} vs {b.gemm_f32.launches}, ms {a.gemm_f32.ms:.3f} vs "
          f"{b.gemm_f32.ms:.3f}", flush=True)
    assert a.gemm_f32.launches == b.gemm_f32.launches > 0
    assert a.gemm_f32.flops == b.gemm_f32.flops
    assert a.matvecs == b.matvecs > 0
    assert 0 < a.gemm_f32.ms < 3 * b.gemm_f32.ms and 0 < b.gemm_f32.ms < 3 * a.gemm_f32.ms
