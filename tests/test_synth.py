"""The seeded generator: determinism, chunk independence and the workload shapes."""
import numpy as np


def test_chunk_and_column_independence(synth_mod):
    cfg = synth_mod.workload("cascadia")
    a = synth_mod.gen_G(cfg, 1000, 12)
    b = np.concatenate([synth_mod.gen_G(cfg, 1007, 5), synth_mod.gen_G(cfg, 1000, 7)][::-1], axis=0)
    assert np.array_equal(a, b)
    cols = np.array([962, 0, 400])
    assert np.array_equal(synth_mod.gen_G(cfg, 1003, 4, cols=cols), a[3:7][:, cols])
    assert np.array_equal(synth_mod.gen_F(cfg, 5, 9), synth_mod.gen_F(cfg, 0, 20)[5:14])
    assert np.array_equal(synth_mod.gen_slip(cfg, 7), synth_mod.gen_slip(cfg, 7))


def test_physical_form_onset_and_decay(synth_mod):
    cfg = synth_mod.workload("small")
    G = synth_mod.gen_G(cfg)
    xs = synth_mod.positions(cfg, "sub"); xg = synth_mod.positions(cfg, "grid")
    d = np.linalg.norm(xg[:, None, :] - xs[None, :, :], axis=-1)
    t = np.arange(cfg.nt) * cfg.dt
    before = t[None, None, :] < (d / cfg.v_g)[:, :, None]
    assert np.all(G[before] == 0)
    # |A| exp(-d/30) bounds the series; A ~ N(0,1) so 6 sigma is generous
    assert np.all(np.abs(G) <= 6.0 * np.exp(-d / cfg.decay_km)[:, :, None] + 1e-7)
    assert (G != 0).mean() > 0.1


def test_slip_pulses(synth_mod):
    for name in ("cascadia", "cascadia_batch"):
        cfg = synth_mod.workload(name)
        xs = synth_mod.positions(cfg, "sub")
        for rup in range(4):
            s, info = synth_mod.gen_slip(cfg, rup, with_info=True)
            act = np.any(s != 0, axis=1)
            assert act.sum() <= info["active"]
            assert s.min() >= 0 and s.max() <= 1
            onset = np.linalg.norm(xs - xs[info["hypocentre"]], axis=1) / cfg.v_rup
            n = np.arange(cfg.nt)[None, :] * cfg.dt
            assert np.all(s[n <= onset[:, None]] == 0)
            if name == "cascadia_batch":
                assert cfg.k_lo <= info["active"] <= cfg.nsub
                assert 2.0 <= info["width_s"] <= 10.0
            else:
                assert 50.0 <= info["extent"] <= 400.0


def test_dense_statistics(synth_mod):
    cfg = synth_mod.workload("small_dense")
    G = synth_mod.gen_G(cfg).astype(np.float64)
    assert abs(G.mean()) < 0.01 and abs(G.std() - 1) < 0.01
    s = synth_mod.gen_slip(cfg, 0)
    assert abs(s.std() - 1) < 0.1
