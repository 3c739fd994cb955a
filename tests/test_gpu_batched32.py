"""Batched float32 path (per-bin complex GEMMs on the matrix cores), through the C-ABI.

Same bar as the single-rupture float32 path: rel-L2 <= 1e-5 per rupture against the FP64
oracle (norm-wise on the tail-dominated physical case), dot-product identity to 1e-6.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import log_case, make_operator, to_dev
from test_gpu_parity import RAGGED, _norm_error_scale

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle_ops(cfg):
    return synth.gen_G(cfg).astype(np.float64), synth.gen_F(cfg).astype(np.float64)


@pytest.mark.parametrize("B", [1, 3, 8, 17, 40, 130])
@pytest.mark.parametrize("diff", [0, 1])
def test_dense_batches(B, diff):
    cfg = synth.workload("small_dense")
    log_case("b32_dense", B=B, diff=diff)
    dt = 0.5
    op = make_operator(cfg, max_batch=B, diff=diff, dt=dt, layout="batched")
    s = synth.gen_slip_batch(cfg, 0, B)
    y = op.forward(to_dev(s)).cpu().numpy()
    G, F = _oracle_ops(cfg)
    errs = oracle.rel_l2_per_rupture(y, oracle.forward(G, F, s, dt=dt, diff=diff))
    print("rel-L2 max", errs.max())
    assert errs.max() <= TOL


def test_small_physical_batched():
    cfg = synth.workload("small")
    log_case("b32_small_physical")
    op = make_operator(cfg, max_batch=8, layout="batched")
    s = synth.gen_slip_batch(cfg, 0, 8)
    y = op.forward(to_dev(s)).cpu().numpy().astype(np.float64)
    G, F = _oracle_ops(cfg)
    yr = oracle.forward(G, F, s)
    scale = _norm_error_scale(G, F, s, cfg.dt)
    for b in range(8):
        err, ny = np.linalg.norm(y[b] - yr[b]), np.linalg.norm(yr[b])
        print(f"rupture {b}: |err| {err:.2e}, rel-L2 {err / ny if ny else float('inf'):.2e}")
        assert err <= TOL * max(scale[b], ny)


@pytest.mark.parametrize("shape", RAGGED, ids=[f"{a}x{b}x{c}x{d}" for a, b, c, d in RAGGED])
def test_ragged_shapes_batched(shape):
    nsub, ngrid, nobs, nt = shape
    cfg = synth.SynthConfig(nsub=nsub, ngrid=ngrid, nobs=nobs, nt=nt, seed=79, slip_seed=80, op_kind="dense",
                            slip_mode="dense")
    log_case("b32_ragged", shape=shape)
    dt = 0.75
    B = 5
    op = make_operator(cfg, max_batch=B, dt=dt, chunk_rows=17, layout="batched")
    s = synth.gen_slip_batch(cfg, 0, B)
    r = synth.normals(6, "r", 0, (B, nobs, nt))
    y = op.forward(to_dev(s)).cpu().numpy()
    gs = op.adjoint(to_dev(r)).cpu().numpy()
    G, F = _oracle_ops(cfg)
    ey = oracle.rel_l2_per_rupture(y, oracle.forward(G, F, s, dt=dt))
    eg = oracle.rel_l2_per_rupture(gs, oracle.adjoint(G, F, r, dt=dt))
    print("forward", ey.max(), "adjoint", eg.max())
    assert ey.max() <= TOL and eg.max() <= TOL


@pytest.mark.parametrize("diff", [0, 1])
def test_adjoint_and_dot_product_batched(diff):
    cfg = synth.workload("small_dense")
    log_case("b32_adjoint_dot", diff=diff)
    dt = 0.5
    B = 12
    op = make_operator(cfg, max_batch=B, diff=diff, dt=dt, layout="batched")
    x = synth.normals(12, "x", 0, (B, cfg.nsub, cfg.nt))
    w = synth.normals(12, "y", 0, (B, cfg.nobs, cfg.nt))
    Ax = op.forward(to_dev(x)).cpu().numpy().astype(np.float64)
    ATw = op.adjoint(to_dev(w)).cpu().numpy().astype(np.float64)
    G, F = _oracle_ops(cfg)
    assert oracle.rel_l2_per_rupture(ATw, oracle.adjoint(G, F, w, dt=dt, diff=diff)).max() <= TOL
    for b in range(B):
        lhs, rhs = np.sum(Ax[b] * w[b]), np.sum(x[b] * ATw[b])
        assert abs(lhs - rhs) <= 1e-6 * np.linalg.norm(Ax[b]) * np.linalg.norm(w[b])


@pytest.mark.parametrize("B", [6, 70])
def test_tile_shapes_bit_identical(B):
    # every tile shape accumulates each output over the same K chunks in the same order
    cfg = synth.SynthConfig(nsub=70, ngrid=300, nobs=20, nt=64, seed=81, slip_seed=82, op_kind="dense",
                            slip_mode="dense")
    log_case("b32_tiles", B=B)
    op = make_operator(cfg, max_batch=B, layout="batched")
    s = to_dev(synth.gen_slip_batch(cfg, 0, B))
    r = to_dev(synth.normals(7, "r", 0, (B, cfg.nobs, cfg.nt)))
    ys, gs = {}, {}
    for c in (1, 2, 3, 4):
        for ck in (1, 2, 3, 4):
            op.set_tuning(gemm32_cfg=c, gemm32_cfg_k=ck, adj32_cfg=ck, gemm32_splits=3, adj32_splits=2)
            ys[c, ck] = op.forward(s).clone()
            gs[c, ck] = op.adjoint(r).clone()
    first = (1, 1)
    for c in ys:
        assert torch.equal(ys[c], ys[first]) and torch.equal(gs[c], gs[first]), f"tile shapes {c} differ"
    G, F = _oracle_ops(cfg)
    assert oracle.rel_l2_per_rupture(ys[first].cpu().numpy(), oracle.forward(G, F, s.cpu().numpy())).max() <= TOL


def test_layouts_agree():
    cfg = synth.workload("small")
    log_case("b32_layouts")
    s = to_dev(synth.gen_slip_batch(cfg, 0, 4))
    y1 = make_operator(cfg, max_batch=4, layout="single").forward(s).cpu().numpy().astype(np.float64)
    y2 = make_operator(cfg, max_batch=4, layout="batched").forward(s).cpu().numpy().astype(np.float64)
    assert np.linalg.norm(y1 - y2) <= 1e-5 * np.linalg.norm(y1)


def test_autograd_batched():
    from paper_2608_21763_amd import source_to_waveform
    cfg = synth.workload("small_dense")
    log_case("b32_autograd")
    B = 9
    op = make_operator(cfg, max_batch=B, layout="batched")
    s_np = synth.gen_slip_batch(cfg, 0, B)
    G, F = _oracle_ops(cfg)
    y_obs = oracle.forward(G, F, synth.gen_slip_batch(cfg, 50, B))
    s = to_dev(s_np).requires_grad_(True)
    loss = 0.5 * ((source_to_waveform(s, op).double() - torch.tensor(y_obs, device="cuda:0")) ** 2).sum()
    loss.backward()
    g = s.grad.cpu().numpy().astype(np.float64)
    g_ref = oracle.adjoint(G, F, oracle.forward(G, F, s_np) - y_obs)
    assert oracle.rel_l2(g, g_ref) <= TOL


@pytest.mark.parametrize("nt", [201, 255])
@pytest.mark.parametrize("layout,dtype", [("batched", "f32"), ("batched", "f16")])
def test_steps_below_256_on_256_bins(nt, layout, dtype):
    # 2 nt padded to 512 gives 256 packed bins, the fused split sum and inverse transform and the
    # register mid-chain, with nt < 256 (odd: the output rows are not 8-byte aligned) and a
    # ragged batch, forward and adjoint
    cfg = synth.SynthConfig(nsub=11, ngrid=70, nobs=9, nt=nt, seed=83, slip_seed=84, op_kind="dense",
                            slip_mode="dense")
    log_case("b32_nt_256_bins", nt=nt, dtype=dtype)
    B = 19
    kw = {"layout": layout} if dtype == "f32" else {"g_dtype": dtype, "f_dtype": dtype}
    op = make_operator(cfg, max_batch=B, dt=0.5, chunk_rows=23, **kw)
    s = synth.gen_slip_batch(cfg, 0, B)
    r = synth.normals(8, "r", 0, (B, cfg.nobs, nt))
    y = op.forward(to_dev(s)).cpu().numpy()
    gs = op.adjoint(to_dev(r)).cpu().numpy()
    G, F = _oracle_ops(cfg)
    ey = oracle.rel_l2_per_rupture(y, oracle.forward(G, F, s, dt=0.5))
    eg = oracle.rel_l2_per_rupture(gs, oracle.adjoint(G, F, r, dt=0.5))
    tol = TOL if dtype == "f32" else 2e-3
    print(dtype, nt, "forward", ey.max(), "adjoint", eg.max())
    assert ey.max() <= tol and eg.max() <= tol


def test_adjoint_tile_control_round_trip():
    # adj32_cfg sets the adjoint's elastic reduction tile on its own: out-of-range ids are
    # refused, and get -> set keeps the public values
    from paper_2608_21763_amd import S2WError
    cfg = synth.workload("small_dense")
    log_case("b32_adj32_cfg")
    op = make_operator(cfg, max_batch=4, layout="batched")
    for bad in (5, -2):
        with pytest.raises(S2WError):
            op.set_tuning(adj32_cfg=bad)
    op.set_tuning(adj32_cfg=2, gemm32_cfg_k=4)
    t = op.get_tuning()
    assert t["adj32_cfg"] == 2 and t["gemm32_cfg_k"] == 4
    op.set_tuning(**t)
    assert op.get_tuning() == t
    op.set_tuning(adj32_cfg=-1)
    assert op.get_tuning()["adj32_cfg"] == -1
