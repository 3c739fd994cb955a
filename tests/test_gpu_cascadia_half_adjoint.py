"""Half-precision adjoint on the Cascadia-shaped share (963 x 37,760 x 64 x 256), bfloat16 and
float16 stores, B = 256 residuals per call: the transpose of the forward map (including D_t's
transpose) against the FP64 oracle's adjoint on sampled residuals and subfault columns, held to
the half-precision bound 2e-3, plus the dot-product identity against the same plan's forward.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import log_case, make_operator, to_dev

pytestmark = pytest.mark.gpu
BOUND = 2e-3


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_half_adjoint_cascadia(dtype):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = synth.workload("cascadia_batch")
    log_case("cascadia_half_adjoint", dtype=dtype, ngrid=cfg.ngrid)
    B = 256
    op = make_operator(cfg, max_batch=B, chunk_rows=1024, g_dtype=dtype, f_dtype=dtype)
    r = synth.normals(cfg.seed, "r", 5, (B, cfg.nobs, cfg.nt))
    gs = op.adjoint(to_dev(r)).cpu().numpy()
    assert np.all(np.isfinite(gs))
    cols = np.array([0, 17, 480, 962])
    rows = [0, 255]
    ref = oracle.adjoint_synth(cfg, r[rows], cols=cols)
    errs = oracle.rel_l2_per_rupture(gs[rows][:, cols, :], ref)
    print(f"{dtype} adjoint rel-L2 on sampled residuals/columns", errs, flush=True)
    assert errs.max() <= BOUND
    x = synth.normals(cfg.seed, "x", 6, (2, cfg.nsub, cfg.nt))
    w = synth.normals(cfg.seed, "y", 6, (2, cfg.nobs, cfg.nt))
    Ax = op.forward(to_dev(x)).cpu().numpy().astype(np.float64)
    ATw = op.adjoint(to_dev(w)).cpu().numpy().astype(np.float64)
    for b in range(2):
        lhs, rhs = np.sum(Ax[b] * w[b]), np.sum(x[b] * ATw[b])
        rel = abs(lhs - rhs) / (np.linalg.norm(Ax[b]) * np.linalg.norm(w[b]))
        print("dot-product mismatch", rel, flush=True)
        assert rel <= BOUND
    del op
    torch.cuda.empty_cache()
