"""The descriptor's limits on every path: all maxima at once (1024 subfaults, 256 observers,
512 steps) and the largest batch (1024 ruptures per call), forward and adjoint, against the FP64
oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import BF16_CEILING, HALF_BOUND, log_case, make_operator, to_dev

pytestmark = pytest.mark.gpu

PATHS = {
    "single": (dict(layout="single"), 1e-5),
    "batched32": (dict(layout="batched"), 1e-5),
    "f16": (dict(g_dtype="f16", f_dtype="f16"), HALF_BOUND),
    # bf16 stores do not meet the 2e-3 bound on dense iid operators: a regression ceiling
    "bf16": (dict(g_dtype="bf16", f_dtype="bf16"), BF16_CEILING),
    "bf16h": (dict(g_dtype="bf16", f_dtype="bf16", products="bf16"), BF16_CEILING),
}


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("path", list(PATHS))
def test_all_maxima(path):
    kw, tol = PATHS[path]
    cfg = synth.SynthConfig(nsub=1024, ngrid=40, nobs=256, nt=512, seed=91, slip_seed=92, op_kind="dense",
                            slip_mode="dense")
    log_case("limits_maxima", path=path)
    op = make_operator(cfg, max_batch=3, **kw)
    s = synth.gen_slip_batch(cfg, 0, 3)
    y = op.forward(to_dev(s)).cpu().numpy()
    G, F = synth.gen_G(cfg).astype(np.float64), synth.gen_F(cfg).astype(np.float64)
    errs = oracle.rel_l2_per_rupture(y, oracle.forward(G, F, s))
    print(path, "rel-L2", errs)
    assert errs.max() <= tol
    r = synth.normals(9, "r", 0, (3, cfg.nobs, cfg.nt))
    g = op.adjoint(to_dev(r)).cpu().numpy()
    eg = oracle.rel_l2_per_rupture(g, oracle.adjoint(G, F, r))
    print(path, "adjoint rel-L2", eg)
    assert eg.max() <= tol


@pytest.mark.parametrize("path", ["batched32", "f16", "bf16", "bf16h"])
def test_largest_batch(path):
    kw, tol = PATHS[path]
    cfg = synth.SynthConfig(nsub=8, ngrid=64, nobs=4, nt=16, seed=93, slip_seed=94, op_kind="dense",
                            slip_mode="dense")
    B = 1024
    log_case("limits_batch", path=path, B=B)
    op = make_operator(cfg, max_batch=B, **kw)
    s = synth.gen_slip_batch(cfg, 0, B)
    y = op.forward(to_dev(s)).cpu().numpy()
    G, F = synth.gen_G(cfg).astype(np.float64), synth.gen_F(cfg).astype(np.float64)
    errs = oracle.rel_l2_per_rupture(y, oracle.forward(G, F, s))
    print(path, "rel-L2 max", errs.max())
    assert errs.max() <= tol
    r = synth.normals(9, "r", 1, (B, cfg.nobs, cfg.nt))
    g = op.adjoint(to_dev(r)).cpu().numpy()
    eg = oracle.rel_l2_per_rupture(g, oracle.adjoint(G, F, r))
    print(path, "adjoint rel-L2 max", eg.max())
    assert eg.max() <= tol


@pytest.mark.parametrize("path", list(PATHS))
def test_empty_batch_every_path(path):
    # B = 0 is a valid call on every layout and store precision: nothing is enqueued and the
    # outputs are empty; a following call still matches the oracle
    kw, tol = PATHS[path]
    cfg = synth.SynthConfig(nsub=9, ngrid=40, nobs=3, nt=20, seed=95, slip_seed=96, op_kind="dense",
                            slip_mode="dense")
    log_case("limits_empty", path=path)
    op = make_operator(cfg, max_batch=4, **kw)
    s0 = torch.empty((0, cfg.nsub, cfg.nt), device="cuda:0")
    r0 = torch.empty((0, cfg.nobs, cfg.nt), device="cuda:0")
    assert op.forward(s0).shape == (0, cfg.nobs, cfg.nt)
    assert op.adjoint(r0).shape == (0, cfg.nsub, cfg.nt)
    s = synth.gen_slip_batch(cfg, 0, 2)
    G, F = synth.gen_G(cfg).astype(np.float64), synth.gen_F(cfg).astype(np.float64)
    assert oracle.rel_l2_per_rupture(op.forward(to_dev(s)).cpu().numpy(), oracle.forward(G, F, s)).max() <= tol


def test_empty_batch_bltt():
    from paper_2608_21763_amd import BLTTOperator
    K = synth.normals(96, "x", 0, (7, 5, 12)).astype(np.float32)
    op = BLTTOperator(7, 5, 12, max_batch=3)
    keep = op.set_blocks(to_dev(K), 0)
    torch.cuda.synchronize()
    del keep
    assert op.apply(torch.empty((0, 5, 12), device="cuda:0")).shape == (0, 7, 12)
    assert op.adjoint(torch.empty((0, 7, 12), device="cuda:0")).shape == (0, 5, 12)
