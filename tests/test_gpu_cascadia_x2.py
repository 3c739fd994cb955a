"""Half-precision stores at a doubled share: 963 x 75,520 x 64 x 256 (about 1/32 of 2,416,530
grid points), bfloat16 and, separately, float16 spectra with per-(grid row, bin) scales,
B in {1, 64}.  The per-rupture rel-L2 against the FP64 oracle is printed for every sampled
rupture (the smallest and the largest active set of the batch and ruptures 0 and 1) and held to
2e-3, with the element-wise error printed beside it.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import log_case, make_operator, to_dev

pytestmark = pytest.mark.gpu
BOUND = 2e-3

_REF = {}


def _ref(cfg, s, b):
    if b not in _REF:
        _REF[b] = oracle.forward_synth(cfg, s[b])
    return _REF[b]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_doubled_share_half(dtype):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = synth.workload("cascadia_x2")
    log_case("cascadia_x2", dtype=dtype, ngrid=cfg.ngrid)
    op = make_operator(cfg, max_batch=64, chunk_rows=1024, g_dtype=dtype, f_dtype=dtype)
    s = synth.gen_slip_batch(cfg, 0, 64)
    act = np.array([np.count_nonzero(np.any(sb != 0, axis=1)) for sb in s])
    y64 = op.forward(to_dev(s)).cpu().numpy()
    y1 = op.forward(to_dev(s[:1])).cpu().numpy()
    picks = sorted({int(np.argmin(act)), int(np.argmax(act)), 0, 1})
    errs = {b: oracle.rel_l2(y64[b], _ref(cfg, s, b)) for b in picks}
    mabs = {b: oracle.max_abs_rel(y64[b], _ref(cfg, s, b)) for b in picks}
    print(f"{dtype} element-wise " + " ".join(f"{b}: {e:.2e}" for b, e in mabs.items()), flush=True)
    e1 = oracle.rel_l2(y1[0], _ref(cfg, s, 0))
    print(f"{dtype}/{dtype} ngrid={cfg.ngrid}: B=64 rel-L2 " +
          " ".join(f"rupture {b} (K={act[b]}): {e:.2e}" for b, e in errs.items()) + f"; B=1 rupture 0: {e1:.2e}",
          flush=True)
    assert max(errs.values()) <= BOUND and e1 <= BOUND and max(mabs.values()) <= BOUND
    del op
    torch.cuda.empty_cache()
