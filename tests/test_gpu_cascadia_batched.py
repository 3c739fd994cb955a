"""Full-size checks of the batched float32 path on the Cascadia-shaped share
(963 x 37,760 x 64 x 256), float32 spectra in the per-bin GEMM layout.

Ensembles: B in {8, 64, 256} ruptures per call, each with its own hypocentre, active set
(K ~ U{20..963} nearest subfaults) and pulse width; rel-L2 <= 1e-5 against the FP64
oracle on sampled ruptures, always including the smallest and largest active sets of the
batch.  Misfit gradient: L = 0.5 * sum_b ||y(s_b) - y_obs||^2 with y_obs the oracle's
waveforms of a hidden rupture plus 1 % Gaussian noise, for B = 64, through the autograd
function; checked against the direct adjoint call, central differences on 20 seeded
coordinates, the dot-product identity and the oracle's adjoint.
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
def batched_op():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = synth.workload("cascadia_batch")
    log_case("cascadia_batched_setup", ngrid=cfg.ngrid)
    op = make_operator(cfg, max_batch=256, chunk_rows=1024, layout="batched")
    yield cfg, op
    del op
    torch.cuda.empty_cache()


def _active(s):
    return np.array([np.count_nonzero(np.any(sb != 0, axis=1)) for sb in s])


@pytest.mark.timeout(900)
def test_forward_ensembles_sampled(batched_op):
    cfg, op = batched_op
    s = synth.gen_slip_batch(cfg, 0, 256)
    act = _active(s)
    ref = {}

    def oracle_of(b):
        if b not in ref:
            ref[b] = oracle.forward_synth(cfg, s[b])
        return ref[b]

    for B in (8, 64, 256):
        picks = sorted({int(np.argmin(act[:B])), int(np.argmax(act[:B])), 0, 1, 2, 3, 4, 5})
        log_case("cascadia_batched_forward", B=B, picks=picks, K=[int(act[b]) for b in picks])
        y = op.forward(to_dev(s[:B])).cpu().numpy()
        errs = [oracle.rel_l2(y[b], oracle_of(b)) for b in picks]
        print(f"B={B} rel-L2 on ruptures {picks}:", " ".join(f"{e:.2e}" for e in errs), flush=True)
        assert max(errs) <= TOL


@pytest.mark.timeout(900)
def test_misfit_gradient_batch64(batched_op):
    from paper_2608_21763_amd import source_to_waveform
    cfg, op = batched_op
    acfg = synth.workload("cascadia_adj")       # same operators, its own ruptures
    B = 64
    log_case("cascadia_batched_gradient", B=B)
    hidden = synth.gen_slip(acfg, 100000)
    y_true = oracle.forward_synth(acfg, hidden)
    rms = np.sqrt(np.mean(y_true ** 2))
    y_obs = y_true + 0.01 * rms * synth.noise(acfg.slip_seed, y_true.shape)
    s_np = synth.gen_slip_batch(acfg, 0, B)
    s = to_dev(s_np).requires_grad_(True)
    y_obs_t = torch.tensor(y_obs, device="cuda:0")
    y = source_to_waveform(s, op)
    loss = 0.5 * ((y.double() - y_obs_t) ** 2).sum()
    loss.backward()
    g = s.grad.cpu().numpy().astype(np.float64)
    # the autograd gradient is the adjoint applied to the residual
    r = (y.detach().double() - y_obs_t).float()
    assert torch.equal(s.grad, op.adjoint(r))
    # central differences of the exactly quadratic loss: every perturbed rupture is one column
    # of a single batched call; the other ruptures' terms cancel exactly
    rng = np.random.default_rng(2608)
    h = 2.0
    coords = [(int(rng.integers(B)), int(rng.integers(cfg.nsub)), int(rng.integers(cfg.nt))) for _ in range(20)]
    pert = np.empty((40, cfg.nsub, cfg.nt), dtype=np.float32)
    for i, (b, j, n) in enumerate(coords):
        pert[2 * i] = s_np[b]
        pert[2 * i, j, n] += h
        pert[2 * i + 1] = s_np[b]
        pert[2 * i + 1, j, n] -= h
    yp = op.forward(to_dev(pert)).cpu().numpy().astype(np.float64)
    gmax = np.abs(g).max()
    worst = 0.0
    for i, (b, j, n) in enumerate(coords):
        lp = 0.5 * np.sum((yp[2 * i] - y_obs) ** 2)
        lm = 0.5 * np.sum((yp[2 * i + 1] - y_obs) ** 2)
        fd = (lp - lm) / (2 * h)
        bound = 1e-3 * abs(g[b, j, n]) + 1e-6 * gmax
        worst = max(worst, abs(fd - g[b, j, n]) / bound)
        assert abs(fd - g[b, j, n]) <= bound, (b, j, n, fd, g[b, j, n])
    print(f"finite differences: worst |fd - g| / bound = {worst:.3f}", flush=True)


@pytest.mark.timeout(900)
def test_adjoint_oracle_and_dot_product(batched_op):
    cfg, op = batched_op
    log_case("cascadia_batched_adjoint")
    B = 64
    r = synth.normals(cfg.seed, "r", 3, (B, cfg.nobs, cfg.nt))
    gs = op.adjoint(to_dev(r)).cpu().numpy()
    cols = np.array([0, 17, 480, 481, 962])
    rows = [0, 21, 42, 63]
    ref = oracle.adjoint_synth(cfg, r[rows], cols=cols)
    errs = oracle.rel_l2_per_rupture(gs[rows][:, cols, :], ref)
    print("adjoint rel-L2 on sampled ruptures/columns", errs, flush=True)
    assert errs.max() <= TOL
    x = synth.normals(cfg.seed, "x", 4, (2, cfg.nsub, cfg.nt))
    w = synth.normals(cfg.seed, "y", 4, (2, cfg.nobs, cfg.nt))
    Ax = op.forward(to_dev(x)).cpu().numpy().astype(np.float64)
    ATw = op.adjoint(to_dev(w)).cpu().numpy().astype(np.float64)
    for b in range(2):
        lhs, rhs = np.sum(Ax[b] * w[b]), np.sum(x[b] * ATw[b])
        rel = abs(lhs - rhs) / (np.linalg.norm(Ax[b]) * np.linalg.norm(w[b]))
        print("dot-product mismatch", rel, flush=True)
        assert rel <= 1e-6
