"""Full-size parity on the Cascadia-shaped share (963 x 37,760 x 64 x 256), float32 spectra.

The oracle evaluates whole ruptures directly in FP64 (only the active subfault
columns are generated; the rest contribute exactly zero).  Adjoint outputs are
checked on sampled subfault columns, which the oracle computes one by one.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import log_case, make_operator, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def cascadia_op():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = synth.workload("cascadia")
    log_case("cascadia_setup", ngrid=cfg.ngrid)
    op = make_operator(cfg, max_batch=4, chunk_rows=1024)
    yield cfg, op
    del op
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
def test_forward_full_share(cascadia_op):
    cfg, op = cascadia_op
    log_case("cascadia_forward", ruptures="0..3")
    s = synth.gen_slip_batch(cfg, 0, 4)
    y = op.forward(to_dev(s)).cpu().numpy()
    yr = oracle.forward_synth(cfg, s)
    errs = oracle.rel_l2_per_rupture(y, yr)
    print("rel-L2 per rupture", errs)
    assert errs.max() <= TOL


@pytest.mark.timeout(600)
def test_adjoint_full_share_sampled_columns(cascadia_op):
    cfg, op = cascadia_op
    log_case("cascadia_adjoint")
    r = synth.normals(cfg.seed, "r", 1, (2, cfg.nobs, cfg.nt))
    gs = op.adjoint(to_dev(r)).cpu().numpy()
    cols = np.array([0, 17, 480, 481, 962])
    ref = oracle.adjoint_synth(cfg, r, cols=cols)
    errs = oracle.rel_l2_per_rupture(gs[:, cols, :], ref)
    print("adjoint rel-L2 on sampled columns", errs)
    assert errs.max() <= TOL


@pytest.mark.timeout(600)
def test_dot_product_full_share(cascadia_op):
    cfg, op = cascadia_op
    log_case("cascadia_dot")
    x = synth.normals(cfg.seed, "x", 2, (2, cfg.nsub, cfg.nt))
    w = synth.normals(cfg.seed, "y", 2, (2, cfg.nobs, cfg.nt))
    Ax = op.forward(to_dev(x)).cpu().numpy().astype(np.float64)
    ATw = op.adjoint(to_dev(w)).cpu().numpy().astype(np.float64)
    for b in range(2):
        lhs, rhs = np.sum(Ax[b] * w[b]), np.sum(x[b] * ATw[b])
        rel = abs(lhs - rhs) / (np.linalg.norm(Ax[b]) * np.linalg.norm(w[b]))
        print("dot-product mismatch", rel)
        assert rel <= 1e-6


@pytest.mark.timeout(600)
def test_displacement_full_share_sampled_rows(cascadia_op):
    # the seafloor displacement from the forward map's own pass, against the oracle's single
    # BLTT of eq. (1) on sampled grid rows; y must not change
    cfg, op = cascadia_op
    log_case("cascadia_displacement", ruptures="0..1")
    s = synth.gen_slip_batch(cfg, 0, 2)
    sd = to_dev(s)
    y_plain = op.forward(sd)
    y, m = op.forward_displacement(sd)
    torch.cuda.synchronize()
    assert torch.equal(y, y_plain)
    rows = np.array([0, 1, 12345, cfg.ngrid // 2, cfg.ngrid - 1])
    Grows = np.stack([synth.gen_G(cfg, int(g), 1)[0] for g in rows]).astype(np.float64)
    ref = oracle.bltt(Grows, s)
    errs = oracle.rel_l2_per_rupture(m.cpu().numpy()[:, rows, :], ref)
    print("displacement rel-L2 on sampled rows", errs, flush=True)
    assert errs.max() <= TOL
    times = [0, 100, 255]
    _, m2 = op.forward_displacement(sd, times)
    torch.cuda.synchronize()
    assert torch.equal(m2, m[:, :, times])
