"""The timed configuration of the measurement line: the Cascadia-shaped share (963 x 37,760 x 64
x 256) with bfloat16 and float16 stores, B = 256 ruptures per call with the default tiles,
against the FP64 oracle on sampled ruptures (the smallest and largest active sets and rupture
0), per-rupture rel-L2 held to the half-precision bound 2e-3 and printed.
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
def test_headline_batch256(dtype):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = synth.workload("cascadia_batch")
    B = 256
    log_case("cascadia_headline", dtype=dtype, B=B)
    op = make_operator(cfg, max_batch=B, chunk_rows=1024, g_dtype=dtype, f_dtype=dtype)
    s = synth.gen_slip_batch(cfg, 0, B)
    y = op.forward(to_dev(s)).cpu().numpy()
    assert np.all(np.isfinite(y))
    act = np.array([np.count_nonzero(np.any(sb != 0, axis=1)) for sb in s])
    picks = sorted({int(np.argmin(act)), int(np.argmax(act)), 0})
    ref = oracle.forward_synth(cfg, s[picks])
    errs = [oracle.rel_l2(y[b], ref[i]) for i, b in enumerate(picks)]
    print(f"{dtype} B={B}: " + " ".join(f"rupture {b} (K={act[b]}): {e:.2e}" for b, e in zip(picks, errs)),
          flush=True)
    assert max(errs) <= BOUND
    del op
    torch.cuda.empty_cache()
