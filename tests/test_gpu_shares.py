"""The paper's other per-GPU shares (Table I) on the float32 single-rupture path:
strong scaling at eight GPUs (60 subfaults x 302,067 grid points x 4 observers) and weak
scaling (480 x 37,758 x 32), 256 steps; rel-L2 <= 1e-5 against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import log_case, make_operator, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["strong_p8", "weak"])
def test_share_forward(name):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = synth.workload(name)
    log_case("share", share=name, nsub=cfg.nsub, ngrid=cfg.ngrid, nobs=cfg.nobs)
    op = make_operator(cfg, max_batch=1, chunk_rows=2048)
    s = synth.gen_slip_batch(cfg, 0, 1)
    y = op.forward(to_dev(s)).cpu().numpy()
    err = oracle.rel_l2(y[0], oracle.forward_synth(cfg, s[0]))
    print(f"{name}: rel-L2 {err:.2e}", flush=True)
    assert err <= TOL
    del op
    torch.cuda.empty_cache()
