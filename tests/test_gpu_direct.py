"""The direct time-domain path (S2W_LAYOUT_DIRECT, eq. 4 form of eqs. 1-2, no FFT) against the oracle.

Float32 on the matrix cores: the bound is the float32 one, rel-L2 <= 1e-5 per rupture, and
because only the kept window's terms enter its sums, it is also held to that plain bound on the
tail-dominated small physical case, where the FFT path's spectral round-off is not (that
path's values are in test_gpu_parity.py).  A rupture whose FP64 reference is exactly zero
gets an absolute bound instead (rel-L2 is undefined there).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import log_case, make_operator, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _ops(cfg):
    return synth.gen_G(cfg).astype(np.float64), synth.gen_F(cfg).astype(np.float64)


def _check(y, yr, what):
    for b in range(y.shape[0]):
        ny = np.linalg.norm(yr[b])
        if ny == 0.0:
            # reference exactly zero: no term of the kept window is nonzero, and none may appear
            amax = float(np.max(np.abs(y[b])))
            print(f"{what} {b}: reference zero, max |y| {amax:.2e}", flush=True)
            assert amax <= 1e-30, amax
            continue
        e = oracle.rel_l2(y[b], yr[b])
        ea = oracle.max_abs_rel(y[b], yr[b])
        print(f"{what} {b}: rel-L2 {e:.3e}, max-abs {ea:.3e}", flush=True)
        assert e <= TOL and ea <= 10 * TOL, (b, e, ea)


def test_direct_small_physical_plain_bound():
    cfg = synth.workload("small")
    log_case("direct_small_physical")
    op = make_operator(cfg, max_batch=4, layout="direct")
    assert op.plan.layout() == "direct"
    s = synth.gen_slip_batch(cfg, 0, 4)
    y = op.forward(to_dev(s)).cpu().numpy().astype(np.float64)
    G, F = _ops(cfg)
    _check(y, oracle.forward(G, F, s), "rupture")


@pytest.mark.parametrize("diff,dt", [(1, 0.5), (0, 1.0), (1, 1.0)])
def test_direct_dense_forward_adjoint(diff, dt):
    cfg = synth.workload("small_dense")
    log_case("direct_dense", diff=diff, dt=dt)
    op = make_operator(cfg, max_batch=3, diff=diff, dt=dt, layout="direct")
    G, F = _ops(cfg)
    s = synth.gen_slip_batch(cfg, 0, 3)
    y = op.forward(to_dev(s)).cpu().numpy().astype(np.float64)
    _check(y, oracle.forward(G, F, s, dt=dt, diff=diff), "forward")
    r = synth.normals(cfg.seed, "r", 0, (3, cfg.nobs, cfg.nt))
    g = op.adjoint(to_dev(r)).cpu().numpy().astype(np.float64)
    _check(g, oracle.adjoint(G, F, r, dt=dt, diff=diff), "adjoint")


RAGGED = [
    # nsub, ngrid, nobs, nt
    (7, 37, 3, 20),
    (1, 1, 1, 1),
    (129, 300, 5, 64),
    (33, 45, 66, 33),        # observers past one 64-row tile
    (300, 131, 2, 100),      # grid rows past one 128-row tile, many channels
    (16, 9, 4, 512),         # longest series: two output ranges of 16 blocks
    (5, 20, 3, 257),         # one step past a single range
]


@pytest.mark.parametrize("shape", RAGGED)
def test_direct_ragged(shape):
    nsub, ngrid, nobs, nt = shape
    cfg = synth.workload("small_dense").replace(nsub=nsub, ngrid=ngrid, nobs=nobs, nt=nt)
    log_case("direct_ragged", shape=shape)
    op = make_operator(cfg, max_batch=2, dt=0.75, layout="direct")
    G, F = _ops(cfg)
    s = synth.gen_slip_batch(cfg, 0, 2)
    y = op.forward(to_dev(s)).cpu().numpy().astype(np.float64)
    _check(y, oracle.forward(G, F, s, dt=0.75), "forward")
    r = synth.normals(cfg.seed, "r", 1, (2, nobs, nt))
    g = op.adjoint(to_dev(r)).cpu().numpy().astype(np.float64)
    _check(g, oracle.adjoint(G, F, r, dt=0.75), "adjoint")


def test_direct_dot_product_and_agreement_with_fft_path():
    # <A x, y> = <x, A^T y> for the direct pair, and the direct and FFT evaluations agree
    cfg = synth.workload("small_dense").replace(nsub=40, ngrid=700, nobs=16, nt=96)
    log_case("direct_dot", shape=(cfg.nsub, cfg.ngrid, cfg.nobs, cfg.nt))
    opd = make_operator(cfg, max_batch=2, layout="direct")
    opf = make_operator(cfg, max_batch=2, layout="single")
    x = synth.normals(cfg.seed, "x", 0, (2, cfg.nsub, cfg.nt))
    w = synth.normals(cfg.seed, "y", 0, (2, cfg.nobs, cfg.nt))
    Ax = opd.forward(to_dev(x)).cpu().numpy().astype(np.float64)
    ATw = opd.adjoint(to_dev(w)).cpu().numpy().astype(np.float64)
    lhs, rhs = float(np.sum(Ax * w)), float(np.sum(x * ATw))
    rel = abs(lhs - rhs) / (np.linalg.norm(Ax) * np.linalg.norm(w))
    print(f"dot: {lhs:.6e} vs {rhs:.6e}, normalised difference {rel:.2e}", flush=True)
    assert rel <= 1e-6
    Af = opf.forward(to_dev(x)).cpu().numpy().astype(np.float64)
    assert oracle.rel_l2(Ax, Af) <= 2 * TOL


def test_direct_empty_batch_and_determinism():
    cfg = synth.workload("small_dense")
    op = make_operator(cfg, max_batch=2, layout="direct")
    s = to_dev(synth.gen_slip_batch(cfg, 0, 2))
    y0 = torch.full((0, cfg.nobs, cfg.nt), 1.0, device="cuda:0")
    op.plan.forward(s.data_ptr(), 0, y0.data_ptr() if y0.numel() else 0, torch.cuda.current_stream().cuda_stream)
    a = op.forward(s)
    b = op.forward(s)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
