"""Plant plausible mistakes in private copies of the oracle and check the pins catch each.

Mistakes in the C source are compiled on the CPU into a temporary library and
checked by the brute-force dense-matrix pins (explicit BLTT block matrices) and
the dot-product identity.  Mistakes in the comparison helpers (rel-L2 and the
element-wise error, on which every parity bound rests) are planted in a copy of
the Python module and checked by the helper pins.  A mutant that survives would
mean the pins cannot tell that mistake from the definition.
"""
import ctypes
import os
import subprocess
import types

import numpy as np
import pytest

from bltt_dense import chain_matrix, to_time_major, from_time_major

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "s2w_oracle.c")
PY_SRC = os.path.join(ROOT, "oracle", "__init__.py")

MUTANTS = {
    "eq1_dropped_last_lag": ("for (int64_t n = k; n < nt; n++) m[n] += gv * sj[n - k];",
                             "for (int64_t n = k + 1; n < nt; n++) m[n] += gv * sj[n - k];"),
    "eq1_shifted_lag": ("for (int64_t n = k; n < nt; n++) m[n] += gv * sj[n - k];",
                        "for (int64_t n = k; n + 1 < nt; n++) m[n + 1] += gv * sj[n - k];"),
    "dt_sign": ("vg[n] = (m[n] - (n > 0 ? m[n - 1] : 0.0)) / dt;",
                "vg[n] = (m[n] + (n > 0 ? m[n - 1] : 0.0)) / dt;"),
    "dt_scale": ("vg[n] = (m[n] - (n > 0 ? m[n - 1] : 0.0)) / dt;",
                 "vg[n] = (m[n] - (n > 0 ? m[n - 1] : 0.0)) * dt;"),
    "dt_first_sample": ("vg[n] = (m[n] - (n > 0 ? m[n - 1] : 0.0)) / dt;",
                        "vg[n] = (m[n] - (n > 0 ? m[n - 1] : m[0])) / dt;"),
    "eq2_wrong_index": ("for (int64_t n = k; n < nt; n++) yo[n] += fv * vg[n - k];",
                        "for (int64_t n = k; n < nt; n++) yo[n] += fv * vg[n];"),
    "eq2_transposed_F": ("const double* fk = F + (g * nobs + o) * nt;\n        const double* vg",
                         "const double* fk = F + (o * nrows + g) * nt;\n        const double* vg"),
    "adj_dropped_lag": ("for (int64_t n = 0; n + k < nt; n++) w[n] += fv * ro[n + k];",
                        "for (int64_t n = 0; n + k < nt - 1; n++) w[n] += fv * ro[n + k];"),
    "adj_dt_direction": ("wg[n] = (w[n] - (n + 1 < nt ? w[n + 1] : 0.0)) / dt;",
                         "wg[n] = (w[n] - (n > 0 ? w[n - 1] : 0.0)) / dt;"),
    "adj_convolution_not_correlation": ("for (int64_t n = 0; n + k < nt; n++) gj[n] += gv * wg[n + k];",
                                        "for (int64_t n = k; n < nt; n++) gj[n] += gv * wg[n - k];"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique in the oracle source"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"lib_{name}.so"
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-std=c99", "-o", str(lib), str(path)], check=True)
    L = ctypes.CDLL(str(lib))
    i64, dbl, i32, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p
    L.s2w_oracle_forward_accum.argtypes = [i64, i64, i64, i64, dbl, i32, vp, vp, i64, vp, vp]
    L.s2w_oracle_adjoint_accum.argtypes = [i64, i64, i64, i64, dbl, i32, vp, vp, i64, vp, vp]
    return L


def _pins_hold(L) -> bool:
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rng = np.random.default_rng(3)
    ngrid, nsub, nobs, nt, dt = 5, 3, 2, 8, 0.5
    G = rng.standard_normal((ngrid, nsub, nt)); F = rng.standard_normal((ngrid, nobs, nt))
    s = rng.standard_normal((1, nsub, nt)); r = rng.standard_normal((1, nobs, nt))
    for diff in (0, 1):
        A = chain_matrix(G, F, dt, diff)
        y = np.zeros((1, nobs, nt)); gs = np.zeros((1, nsub, nt))
        L.s2w_oracle_forward_accum(ngrid, nsub, nobs, nt, dt, diff, p(G), p(F), 1, p(s), p(y))
        L.s2w_oracle_adjoint_accum(ngrid, nsub, nobs, nt, dt, diff, p(G), p(F), 1, p(r), p(gs))
        if not np.allclose(y[0], from_time_major(A @ to_time_major(s[0]), nobs), rtol=1e-10, atol=1e-10):
            return False
        if not np.allclose(gs[0], from_time_major(A.T @ to_time_major(r[0]), nsub), rtol=1e-10, atol=1e-10):
            return False
        if abs(np.sum(y * r) - np.sum(s * gs)) > 1e-10 * np.linalg.norm(y) * np.linalg.norm(r):
            return False
    return True


def test_unmutated_source_passes(tmp_path):
    src = open(SRC).read()
    L = _build(tmp_path, "clean", src[:40], src[:40])
    assert _pins_hold(L)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    L = _build(tmp_path, name, old, new)
    assert not _pins_hold(L), f"planted mistake '{name}' survived the pins"


# planted mistakes in the comparison helpers of the Python module
HELPER_MUTANTS = {
    "rel_l2_squared_ratio": ("return float(np.sqrt(np.sum((y - yref) ** 2)) / den) if den > 0",
                             "return float(np.sum((y - yref) ** 2) / den ** 2) if den > 0"),
    "rel_l2_result_denominator": ("den = np.sqrt(np.sum(yref * yref))",
                                  "den = np.sqrt(np.sum(y * y))"),
    "rel_l2_sum_denominator": ("den = np.sqrt(np.sum(yref * yref))",
                               "den = np.sqrt(np.sum(yref * yref) + np.sum(y * y))"),
    "rel_l2_zero_reference_passes": ("else float(np.sqrt(np.sum(y * y)))", "else 0.0"),
    "rel_l2_no_square_root": ("return float(np.sqrt(np.sum((y - yref) ** 2)) / den) if den > 0",
                              "return float(np.sum(np.abs(y - yref)) / den) if den > 0"),
    "per_rupture_pooled": ("np.array([rel_l2(y[b], yref[b]) for b in range(y.shape[0])])",
                           "np.array([rel_l2(y, yref) for b in range(y.shape[0])])"),
    "max_abs_mean_not_max": ("num = float(np.max(np.abs(y - yref))) if y.size else 0.0",
                             "num = float(np.mean(np.abs(y - yref))) if y.size else 0.0"),
    "max_abs_result_denominator": ("den = float(np.max(np.abs(yref))) if yref.size else 0.0",
                                   "den = float(np.max(np.abs(y))) if yref.size else 0.0"),
}


def _helper_module(name, old, new):
    src = open(PY_SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique in the oracle module"
    ns = {"__name__": f"oracle_mutant_{name}", "__file__": PY_SRC}
    exec(compile(src.replace(old, new), f"<{name}>", "exec"), ns)
    return types.SimpleNamespace(**ns)


def test_unmutated_helpers_pass():
    from metric_pins import failures
    assert failures(_helper_module("clean", "import ctypes", "import ctypes")) == []


@pytest.mark.parametrize("name", sorted(HELPER_MUTANTS))
def test_helper_mutant_is_caught(name):
    from metric_pins import failures
    old, new = HELPER_MUTANTS[name]
    assert failures(_helper_module(name, old, new)), f"planted mistake '{name}' survived the helper pins"
