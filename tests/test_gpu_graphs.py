"""Replayed HIP graphs for lbm_step (lbm_set_graphs) give the same state, inlet plane
and statistics as plain launches, bit for bit, across batches, a remainder, a
changed kernel argument (C_s) and a changed state buffer (GPU tests)."""
import numpy as np
import pytest
import torch

from parity_cases import Case

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _run(case, graphs, planes):
    ch = case.ch
    ch.set_graphs(graphs)
    ch.stats_attach(planes)
    ch.step(70)                 # two graph batches and a remainder of 6
    ch.set_cs_smag(0.13)        # a changed kernel argument invalidates the graphs
    ch.step(64)
    f, h = ch.state()
    f0, h0 = f.clone(), h.clone()
    t0 = ch.time
    ch.step(33)
    ch.set_state(f0, h0, t0)    # back to a saved state in other buffers
    ch.step(40)
    ch.sync()
    means, n = ch.stats_read()
    u_in = ch.u_in.clone() if case.xbc == "inflow" else None
    return ch.populations().cpu(), ch.state()[1].cpu(), means, n, u_in, ch.time


@pytest.mark.parametrize("kw,storage", [
    (dict(ywall="slip", xbc="inflow", wall_model=True), "f32"),
    (dict(ywall="slip", xbc="inflow", wall_model=True), "f16dev"),
    (dict(ywall="bounceback", xbc="periodic", wall_model=True, g=(4e-6, 0.0, 0.0), wall_avg="line"), "f16dev"),
])
def test_graph_replay_matches_plain_launches(kw, storage):
    _say("graphs", kw, storage)
    out = {}
    for graphs in (False, True):
        case = Case(7, 10, 70, storage=storage, **kw)
        out[graphs] = _run(case, graphs, [2, 5])
        case.ch.close()
    a, b = out[False], out[True]
    assert torch.equal(a[0], b[0])
    if kw["xbc"] == "inflow":
        assert torch.equal(a[1], b[1]) and torch.equal(a[4], b[4])
    assert np.array_equal(a[2], b[2]) and a[3] == b[3] and a[5] == b[5]
