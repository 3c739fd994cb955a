"""One block lower-triangular Toeplitz operator on its own (Alg. 2), through the C-ABI.

Parity with the FP64 oracle's single BLTT matvec (rel-L2 <= 1e-5 per history), the
dot-product identity, the composition with D_t that reproduces the two-operator map, and the
seafloor displacement of a full Cascadia-sized share on sampled grid rows.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import log_case, make_operator, to_dev
from paper_2608_21763_amd import BLTTOperator

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bltt_op(K, max_batch):
    op = BLTTOperator(K.shape[0], K.shape[1], K.shape[2], max_batch=max_batch)
    keep = op.set_blocks(to_dev(K), 0)
    torch.cuda.synchronize()
    del keep
    return op


SHAPES = [
    # nrow, ncol, nt
    (300, 40, 64),     # tall: many output rows (elastic-like)
    (6, 700, 32),      # wide: few output rows, long reduction (acoustic-like)
    (7, 13, 20),
    (1, 1, 1),
    (16, 9, 512),
    (64, 3000, 256),
]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{a}x{b}x{c}" for a, b, c in SHAPES])
@pytest.mark.parametrize("B", [1, 2, 3, 5, 70])
def test_apply_and_adjoint_match_oracle(shape, B):
    nrow, ncol, nt = shape
    log_case("bltt", shape=shape, B=B)
    K = synth.normals(21, "x", nrow * 7 + ncol, (nrow, ncol, nt)).astype(np.float32)
    x = synth.normals(21, "y", B, (B, ncol, nt)).astype(np.float32)
    r = synth.normals(21, "r", B, (B, nrow, nt)).astype(np.float32)
    op = _bltt_op(K, B)
    y = op.apply(to_dev(x)).cpu().numpy().astype(np.float64)
    g = op.adjoint(to_dev(r)).cpu().numpy().astype(np.float64)
    ey = oracle.rel_l2_per_rupture(y, oracle.bltt(K, x))
    eg = oracle.rel_l2_per_rupture(g, oracle.bltt(K, r, trans=True))
    print("apply", ey.max(), "adjoint", eg.max())
    assert ey.max() <= TOL and eg.max() <= TOL
    for b in range(min(B, 4)):
        lhs, rhs = np.sum(y[b] * r[b]), np.sum(x[b] * g[b])
        assert abs(lhs - rhs) <= 1e-6 * np.linalg.norm(y[b]) * np.linalg.norm(r[b])


def test_composition_reproduces_the_map():
    # elastic operator (rows = grid points) -> D_t -> acoustic operator (rows = observers)
    cfg = synth.workload("small")
    log_case("bltt_composition")
    G = synth.gen_G(cfg)                                   # [g][j][k]
    F = synth.gen_F(cfg)                                   # [g][o][k]
    Fq = np.ascontiguousarray(np.transpose(F, (1, 0, 2)))  # [o][g][k]
    s = to_dev(synth.gen_slip_batch(cfg, 0, 3))
    elastic = _bltt_op(G, 3)
    acoustic = _bltt_op(Fq, 3)
    m = elastic.apply(s)                                   # seafloor displacement [b][g][n]
    v = (m - torch.nn.functional.pad(m, (1, 0))[:, :, :-1]) / cfg.dt
    y_chain = acoustic.apply(v).cpu().numpy().astype(np.float64)
    y_map = make_operator(cfg, max_batch=3).forward(s).cpu().numpy().astype(np.float64)
    assert np.linalg.norm(y_chain - y_map) <= 1e-5 * np.linalg.norm(y_map)
    m_ref = oracle.bltt(G, s.cpu().numpy())
    assert oracle.rel_l2(m.cpu().numpy(), m_ref) <= TOL


@pytest.mark.timeout(600)
def test_seafloor_displacement_full_share():
    # the elastic operator of the Cascadia-sized share on its own: displacement of every grid
    # row for one rupture, checked on sampled rows
    cfg = synth.workload("cascadia")
    log_case("bltt_cascadia_displacement", ngrid=cfg.ngrid)
    op = BLTTOperator(cfg.ngrid, cfg.nsub, cfg.nt, max_batch=2)
    op.load_blocks(lambda r0, n, out: synth.gen_G(cfg, r0, n, out=out), chunk_rows=512)
    s = synth.gen_slip_batch(cfg, 0, 2)
    m = op.apply(to_dev(s)).cpu().numpy()
    rows = np.array([0, 1, 4095, 20000, cfg.ngrid - 1])
    Gs = np.stack([synth.gen_G(cfg, int(g), 1)[0] for g in rows])
    ref = oracle.bltt(Gs, s)
    errs = oracle.rel_l2_per_rupture(m[:, rows, :], ref)
    print("displacement rel-L2 on sampled rows", errs)
    assert errs.max() <= TOL
