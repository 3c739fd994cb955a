"""Forward and adjoint calls captured into a HIP graph (through torch.cuda.graph) and replayed.

Each replay must reproduce the eager result bit for bit, with eager calls of the same plan
(which reuse its workspace) and synchronisations in between, and must pick up new input
values written into the captured buffers.  Also: the autotuner picks a shape without
changing the numbers.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import log_case, make_operator, to_dev

pytestmark = pytest.mark.gpu

KINDS = {
    "single": dict(layout="single"),
    "batched32": dict(layout="batched"),
    "half": dict(g_dtype="bf16", f_dtype="bf16"),
    "half_bf16_products": dict(g_dtype="bf16", f_dtype="bf16", products="bf16"),
    "half16": dict(g_dtype="f16", f_dtype="f16"),
}


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _capture(fn):
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()                       # warm-up on the capturing stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("kind", list(KINDS))
def test_graph_replays_match_eager(kind):
    cfg = synth.SynthConfig(nsub=40, ngrid=300, nobs=12, nt=64, seed=83, slip_seed=84, op_kind="dense",
                            slip_mode="dense")
    B = 5
    log_case("graph", kind=kind, B=B)
    op = make_operator(cfg, max_batch=B, **KINDS[kind])
    s = to_dev(synth.gen_slip_batch(cfg, 0, B))
    s2 = to_dev(synth.gen_slip_batch(cfg, 10, B))
    y = torch.empty((B, cfg.nobs, cfg.nt), device="cuda:0")
    eager = op.forward(s).clone()
    eager2 = op.forward(s2).clone()
    g = _capture(lambda: op.forward(s, out=y))
    for k in range(3):
        y.zero_()
        other = op.forward(s2)          # eager use of the same workspace between replays
        torch.cuda.synchronize()
        assert torch.equal(other, eager2)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, eager), f"replay {k}"
    s.copy_(s2)
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(y, eager2)
    # every path's adjoint replays too
    r = to_dev(synth.normals(8, "r", 0, (B, cfg.nobs, cfg.nt)))
    gs = torch.empty((B, cfg.nsub, cfg.nt), device="cuda:0")
    adj = op.adjoint(r).clone()
    ga = _capture(lambda: op.adjoint(r, out=gs))
    for k in range(3):
        gs.zero_()
        op.forward(s2)
        torch.cuda.synchronize()
        ga.replay()
        torch.cuda.synchronize()
        assert torch.equal(gs, adj), f"adjoint replay {k}"


@pytest.mark.parametrize("kind", list(KINDS))
def test_autotune_keeps_results(kind, tmp_path):
    from paper_2608_21763_amd import autotune
    cfg = synth.SynthConfig(nsub=70, ngrid=400, nobs=20, nt=64, seed=85, slip_seed=86, op_kind="dense",
                            slip_mode="dense")
    B = 24
    log_case("autotune", kind=kind, B=B)
    op = make_operator(cfg, max_batch=B, **KINDS[kind])
    if kind == "batched32":
        op.set_tuning(gemm32_splits=2, adj32_splits=2)    # fixed split counts: shapes alone vary
    elif kind != "single":
        op.set_tuning(adj32_splits=2)
    s = to_dev(synth.gen_slip_batch(cfg, 0, B))
    r = to_dev(synth.normals(cfg.seed, "r", 0, (B, cfg.nobs, cfg.nt)))
    y0 = op.forward(s).clone()
    g0 = op.adjoint(r).clone()
    cache = str(tmp_path / "tune.json")
    res = autotune(op, B, reps=2, cache_path=cache)
    assert not res["cached"] and len(res["results"]) > 1
    print(kind, "best", res["best"], f"{res['ms']:.3f} ms")
    y1 = op.forward(s)
    if kind == "single":
        np.testing.assert_allclose(y1.cpu().numpy(), y0.cpu().numpy(), rtol=0, atol=1e-5 * float(y0.abs().max()))
    else:
        assert torch.equal(y1, y0)
        assert torch.equal(op.adjoint(r), g0)
    again = autotune(op, B, cache_path=cache)
    assert again["cached"] and again["best"] == res["best"]


@pytest.mark.parametrize("B", [1, 6])
def test_bltt_graph_replays(B):
    # the standalone operator's apply (matrix-vector kernel for B <= 4, matrix cores beyond)
    # and adjoint replay from a captured graph with the eager results
    from paper_2608_21763_amd import BLTTOperator
    nrow, ncol, nt = 50, 30, 40
    K = synth.normals(87, "x", 0, (nrow, ncol, nt)).astype(np.float32)
    op = BLTTOperator(nrow, ncol, nt, max_batch=B)
    keep = op.set_blocks(to_dev(K), 0)
    torch.cuda.synchronize()
    del keep
    x = to_dev(synth.normals(87, "y", 0, (B, ncol, nt)))
    r = to_dev(synth.normals(87, "r", 0, (B, nrow, nt)))
    y = torch.empty((B, nrow, nt), device="cuda:0")
    g = torch.empty((B, ncol, nt), device="cuda:0")
    ye, ge = op.apply(x).clone(), op.adjoint(r).clone()
    graph = _capture(lambda: (op.apply(x, out=y), op.adjoint(r, out=g)))
    for k in range(3):
        y.zero_()
        g.zero_()
        op.apply(x)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ye) and torch.equal(g, ge), f"replay {k}"
