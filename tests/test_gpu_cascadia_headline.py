"""The timed configuration of the measurement line: the Cascadia-shaped share (963 x 37,760 x 64
x 256) with bfloat16 and float16 stores, B = 256 ruptures per call with the default tiles,
against the FP64 oracle on 34 sampled ruptures of the batch (every eighth, plus the smallest
and the largest active set).

The oracle's waveforms for those ruptures are stored in tests/golden/headline_ref.npz, written
by tests/golden/make_headline_ref.py, which calls only the oracle and the seeded generator (a
whole run of the oracle over 34 ruptures of this share takes tens of minutes of CPU time).
Per-rupture rel-L2 and element-wise errors are printed (max, p95, median).  Float16 stores and
the timed store (bfloat16 elastic, float16 acoustic spectra) are held to the half-precision bound
2e-3 on every sampled rupture (measured max 3.4e-4 and 1.70e-3).  Bfloat16 stores for both
operators do NOT meet 2e-3 on every sampled rupture (measured max 2.15e-3 on rupture 56, p95
1.90e-3, median 1.59e-3): they are held to the regression ceiling gpu_util.BF16_CEILING and the
printed line says whether 2e-3 is met.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import HALF_BOUND, half_limit, log_case, make_operator, report_half, to_dev

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "headline_ref.npz")


def headline_reference():
    d = np.load(GOLDEN, allow_pickle=False)
    return d["indices"], d["active"], d["y"].astype(np.float64)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtypes", [("bf16", "bf16", "auto"), ("bf16", "bf16", "bf16"), ("f16", "f16", "auto"),
                                    ("bf16", "f16", "auto")])
def test_headline_batch256(dtypes):
    gdt, fdt, products = dtypes
    dtype = f"{gdt}/{fdt}" + (" bf16 products" if products == "bf16" else "")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = synth.workload("cascadia_batch")
    B = 256
    idx, act, ref = headline_reference()
    log_case("cascadia_headline", dtype=dtype, B=B, sampled=len(idx))
    s = synth.gen_slip_batch(cfg, 0, B)
    act_now = np.array([np.count_nonzero(np.any(s[b] != 0, axis=1)) for b in idx])
    assert np.array_equal(act_now, act), "the stored reference is for another batch"
    assert act.min() == min(np.count_nonzero(np.any(sb != 0, axis=1)) for sb in s)
    op = make_operator(cfg, max_batch=B, chunk_rows=1024, g_dtype=gdt, f_dtype=fdt, products=products)
    y = op.forward(to_dev(s)).cpu().numpy()
    assert np.all(np.isfinite(y))
    rel = np.array([oracle.rel_l2(y[b], ref[i]) for i, b in enumerate(idx)])
    mabs = np.array([oracle.max_abs_rel(y[b], ref[i]) for i, b in enumerate(idx)])
    worst = int(np.argmax(rel))
    print(f"{dtype} B={B}, {len(idx)} ruptures: rel-L2 max {rel.max():.3e} (rupture {idx[worst]}, K={act[worst]}), "
          f"p95 {np.percentile(rel, 95):.3e}, median {np.median(rel):.3e}; min-K rupture {idx[np.argmin(act)]} "
          f"{rel[np.argmin(act)]:.3e}, max-K rupture {idx[np.argmax(act)]} {rel[np.argmax(act)]:.3e}", flush=True)
    report_half(f"{dtype} B={B}", rel, mabs)
    # the timed store meets the bound on this workload (not on dense iid operators, where the
    # bfloat16 elastic store alone adds about as much rounding: tests/test_gpu_half.py)
    limit = HALF_BOUND if (gdt, fdt) == ("bf16", "f16") else half_limit(gdt, fdt)
    assert rel.max() <= limit and mabs.max() <= limit
    del op
    torch.cuda.empty_cache()
