"""Seafloor displacement from the forward map's own pass (s2w_forward_displacement).

m[b][g][i] is eq. (1) at grid row g and step times[i]: one block lower-triangular Toeplitz
product of the elastic blocks with the slip rate, which the oracle's single-BLTT evaluation
(`oracle.bltt`) computes directly in FP64.  On every layout the waveforms must equal
s2w_forward's bit for bit, and m must match the oracle at the path's bound: rel-L2 1e-5 for
float32 stores, 2e-3 for half-precision stores (whose elastic blocks are rounded).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import log_case, make_operator, to_dev
from paper_2608_21763_amd import S2WError

pytestmark = pytest.mark.gpu

CASES = [
    # layout, dtype, (nsub, ngrid, nobs, nt), B
    ("single", "f32", (16, 512, 4, 32), 2),
    ("single", "f32", (7, 203, 4, 33), 1),         # L = 128
    ("single", "f32", (7, 203, 70, 200), 1),       # 70 observers at L = 512: the unfused kernels
    ("batched", "f32", (16, 300, 4, 32), 9),
    ("batched", "f32", (21, 70, 5, 256), 19),      # M = 256: the register mid-chain, ragged rupture block
    ("batched", "bf16", (16, 300, 4, 32), 9),
    ("batched", "f16", (21, 70, 5, 256), 19),
    ("direct", "f32", (16, 512, 4, 32), 2),
    ("direct", "f32", (5, 150, 3, 300), 2),        # two output ranges
]


def _bound(dtype):
    return 1e-5 if dtype == "f32" else 2e-3


@pytest.mark.parametrize("layout,dtype,shape,B", CASES)
@pytest.mark.parametrize("sel", ["all", "some"])
def test_displacement_matches_oracle(layout, dtype, shape, B, sel):
    nsub, ngrid, nobs, nt = shape
    cfg = synth.workload("small_dense").replace(nsub=nsub, ngrid=ngrid, nobs=nobs, nt=nt)
    log_case("displacement", layout=layout, dtype=dtype, shape=shape, B=B, sel=sel)
    kw = {} if dtype == "f32" else {"g_dtype": dtype, "f_dtype": dtype}
    op = make_operator(cfg, max_batch=B, dt=0.5, layout=layout, **kw)
    s_np = synth.gen_slip_batch(cfg, 0, B)
    s = to_dev(s_np)
    times = None if sel == "all" else sorted({0, 1, nt // 3, nt // 2 + 1, nt - 1})
    y_ref_gpu = op.forward(s)
    y, m = op.forward_displacement(s, times)
    torch.cuda.synchronize()
    assert torch.equal(y, y_ref_gpu), "waveforms differ from s2w_forward"
    cols = np.arange(nt) if times is None else np.array(times)
    G = synth.gen_G(cfg).astype(np.float64)
    m_ref = oracle.bltt(G, s_np)[:, :, cols]                    # [B][ngrid][ntimes]
    m = m.cpu().numpy().astype(np.float64)
    assert m.shape == m_ref.shape
    e = oracle.rel_l2_per_rupture(m, m_ref)
    ea = oracle.max_abs_rel_per_rupture(m, m_ref)
    print(f"{layout}/{dtype} {shape} B={B} {sel}: m rel-L2 max {e.max():.2e}, max-abs {ea.max():.2e}", flush=True)
    assert e.max() <= _bound(dtype) and ea.max() <= 10 * _bound(dtype)


def test_displacement_time_lists_validated():
    cfg = synth.workload("small_dense")
    op = make_operator(cfg, max_batch=1, layout="single")
    s = to_dev(synth.gen_slip_batch(cfg, 0, 1))
    y = torch.empty((1, cfg.nobs, cfg.nt), device="cuda:0")
    m = torch.empty((1, cfg.ngrid, cfg.nt), device="cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    for times, n in [([3, 3], 2), ([5, 2], 2), ([-1], 1), ([cfg.nt], 1), (None, cfg.nt - 1), ([], 0)]:
        with pytest.raises(S2WError) as ei:
            op.plan.forward_displacement(s.data_ptr(), 1, y.data_ptr(), m.data_ptr(), times, n, st)
        assert ei.value.code == "S2W_EINVAL", (times, n)
    with pytest.raises(S2WError):
        op.plan.forward_displacement(s.data_ptr(), 1, y.data_ptr(), y.data_ptr(), None, cfg.nt, st)
    # the last step alone
    y1, m1 = op.forward_displacement(s, [cfg.nt - 1])
    _, mall = op.forward_displacement(s, None)
    torch.cuda.synchronize()
    assert torch.equal(m1[:, :, 0], mall[:, :, cfg.nt - 1])
