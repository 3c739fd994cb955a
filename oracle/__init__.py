"""FP64 CPU oracle for the source-to-waveform map -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_2608_21763_amd``) and never imports it; both draw inputs from
the seeded generator in ``synth``.

What it computes (``s2w_oracle.c``): the paper's direct time-domain
definitions in double precision -- eq. (1) elastic response, the temporal
difference D_t (Sec. II-B2), eq. (2) waveform response, each convolution in
the channel form of eq. (4) -- giving one share's term of eq. (3), and the
exact transpose of that map.  No FFT anywhere.

Readings where the paper is silent: D_t is the backward difference
(m_n - m_{n-1})/dt with m_{-1} = 0 (``diff=1``), or the identity
(``diff=0``); lag k = 0 is the same-step response.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libs2w_oracle.so")
_SRC = os.path.join(_HERE, "s2w_oracle.c")

DIFF_NONE = 0
DIFF_BACKWARD = 1


def build(verbose: bool = False) -> str:
    """Compile the oracle into ``libs2w_oracle.so`` (gcc, OpenMP, FP64)."""
    cmd = ["gcc", "-O3", "-mavx2", "-mfma", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall", "-o", _LIB_PATH + ".tmp", _SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, dbl, i32, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p
        lib.s2w_oracle_forward_accum.argtypes = [i64, i64, i64, i64, dbl, i32, vp, vp, i64, vp, vp]
        lib.s2w_oracle_adjoint_accum.argtypes = [i64, i64, i64, i64, dbl, i32, vp, vp, i64, vp, vp]
        lib.s2w_oracle_bltt.argtypes = [i64, i64, i64, vp, i64, i32, vp, vp]
        _lib = lib
    return _lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def forward(G, F, s, dt: float = 1.0, diff: int = DIFF_BACKWARD) -> np.ndarray:
    """y[b][o][n] for G[g][j][k], F[g][o][k], s[b][j][n] (or s[j][n]); float64."""
    G, F, s = _d(G), _d(F), _d(s)
    squeeze = s.ndim == 2
    if squeeze:
        s = s[None]
    ngrid, nsub, nt = G.shape
    nobs = F.shape[1]
    assert F.shape == (ngrid, nobs, nt) and s.shape[1:] == (nsub, nt)
    y = np.zeros((s.shape[0], nobs, nt))
    _load().s2w_oracle_forward_accum(ngrid, nsub, nobs, nt, dt, diff, _p(G), _p(F), s.shape[0], _p(s), _p(y))
    return y[0] if squeeze else y


def adjoint(G, F, r, dt: float = 1.0, diff: int = DIFF_BACKWARD) -> np.ndarray:
    """gs[b][j][n] = (A^T r)[b] for r[b][o][n] (or r[o][n]); float64."""
    G, F, r = _d(G), _d(F), _d(r)
    squeeze = r.ndim == 2
    if squeeze:
        r = r[None]
    ngrid, nsub, nt = G.shape
    nobs = F.shape[1]
    assert F.shape == (ngrid, nobs, nt) and r.shape[1:] == (nobs, nt)
    gs = np.zeros((r.shape[0], nsub, nt))
    _load().s2w_oracle_adjoint_accum(ngrid, nsub, nobs, nt, dt, diff, _p(G), _p(F), r.shape[0], _p(r), _p(gs))
    return gs[0] if squeeze else gs


def bltt(K, x, trans: bool = False) -> np.ndarray:
    """One causal block-Toeplitz matvec in the form of eq. (4), K[i][j][k] = [F_k]_{ij}.

    trans=False: x[b][j][n] -> y[b][i][n];  trans=True: y[b][i][n] -> x[b][j][n].
    """
    K, x = _d(K), _d(x)
    squeeze = x.ndim == 2
    if squeeze:
        x = x[None]
    nout, nin, nt = K.shape
    B = x.shape[0]
    out = np.zeros((B, nin if trans else nout, nt))
    assert x.shape[1:] == ((nout if trans else nin), nt)
    _load().s2w_oracle_bltt(nout, nin, nt, _p(K), B, int(trans), _p(x), _p(out))
    return out[0] if squeeze else out


def _chunks(n: int, size: int):
    for r0 in range(0, n, size):
        yield r0, min(size, n - r0)


class _ChunkBuffers:
    """Reusable host buffers for operator chunks (fresh allocations page-fault slowly)."""

    def __init__(self):
        self.bufs = {}

    def get(self, key, shape, dtype):
        b = self.bufs.get(key)
        n = int(np.prod(shape))
        if b is None or b.size < n or b.dtype != dtype:
            b = np.empty(n, dtype=dtype)
            self.bufs[key] = b
        return b[:n].reshape(shape)


_BUF = _ChunkBuffers()


def _operator_chunk(cfg, r0, nr, cols):
    import synth
    g32 = _BUF.get("g32", (nr, len(cols), cfg.nt), np.float32)
    f32 = _BUF.get("f32", (nr, cfg.nobs, cfg.nt), np.float32)
    synth.gen_G(cfg, r0, nr, cols=cols, out=g32)
    synth.gen_F(cfg, r0, nr, out=f32)
    G = _BUF.get("g64", g32.shape, np.float64)
    F = _BUF.get("f64", f32.shape, np.float64)
    np.copyto(G, g32)
    np.copyto(F, f32)
    return G, F


def forward_synth(cfg, s, dt: float | None = None, diff: int = DIFF_BACKWARD, chunk_rows: int = 512) -> np.ndarray:
    """Forward map over a whole synthetic share, operators regenerated in grid-row chunks.

    Only subfault columns where some rupture in ``s`` is nonzero are generated
    (the others contribute exactly zero).  The operators are the generator's
    float32 values promoted to float64: the same numbers the GPU receives.
    """
    import synth
    s = _d(s)
    squeeze = s.ndim == 2
    if squeeze:
        s = s[None]
    dt = cfg.dt if dt is None else dt
    cols = synth.active_columns(s)
    sa = np.ascontiguousarray(s[:, cols, :])
    B = s.shape[0]
    y = np.zeros((B, cfg.nobs, cfg.nt))
    lib = _load()
    if len(cols):
        for r0, nr in _chunks(cfg.ngrid, chunk_rows):
            G, F = _operator_chunk(cfg, r0, nr, cols)
            lib.s2w_oracle_forward_accum(nr, len(cols), cfg.nobs, cfg.nt, dt, diff, _p(G), _p(F), B, _p(sa), _p(y))
    return y[0] if squeeze else y


def adjoint_synth(cfg, r, cols=None, dt: float | None = None, diff: int = DIFF_BACKWARD,
                  chunk_rows: int = 512) -> np.ndarray:
    """Adjoint over a whole synthetic share for the subfault columns ``cols`` (default all).

    Returns gs[b][q][n] for j = cols[q].
    """
    r = _d(r)
    squeeze = r.ndim == 2
    if squeeze:
        r = r[None]
    dt = cfg.dt if dt is None else dt
    cols = np.arange(cfg.nsub, dtype=np.int64) if cols is None else np.asarray(cols, dtype=np.int64)
    B = r.shape[0]
    gs = np.zeros((B, len(cols), cfg.nt))
    lib = _load()
    for r0, nr in _chunks(cfg.ngrid, chunk_rows):
        G, F = _operator_chunk(cfg, r0, nr, cols)
        lib.s2w_oracle_adjoint_accum(nr, len(cols), cfg.nobs, cfg.nt, dt, diff, _p(G), _p(F), B, _p(r), _p(gs))
    return gs[0] if squeeze else gs


def rel_l2(y, yref) -> float:
    """||y - yref||_2 / ||yref||_2 over every entry, accumulated in float64.

    The denominator is the reference's norm, never the tested result's.  When the
    reference is identically zero there is nothing to be relative to: the value
    returned is then the absolute norm ||y||_2, and a caller bounds it with an
    absolute bound of its own.
    """
    y, yref = _d(y), _d(yref)
    den = np.sqrt(np.sum(yref * yref))
    return float(np.sqrt(np.sum((y - yref) ** 2)) / den) if den > 0 else float(np.sqrt(np.sum(y * y)))


def rel_l2_per_rupture(y, yref) -> np.ndarray:
    """rel-L2 of each rupture (leading axis) over its own (o, n) entries."""
    y, yref = _d(y), _d(yref)
    return np.array([rel_l2(y[b], yref[b]) for b in range(y.shape[0])])


def max_abs_rel(y, yref) -> float:
    """Element-wise error max |y - yref| / max |yref|, in float64.

    Unlike rel-L2, one wrong sample cannot hide in a large norm: it shows at its
    full size.  A zero reference gives the absolute max |y|, as in rel_l2.
    """
    y, yref = _d(y), _d(yref)
    den = float(np.max(np.abs(yref))) if yref.size else 0.0
    num = float(np.max(np.abs(y - yref))) if y.size else 0.0
    return num / den if den > 0 else (float(np.max(np.abs(y))) if y.size else 0.0)


def max_abs_rel_per_rupture(y, yref) -> np.ndarray:
    """max_abs_rel of each rupture (leading axis) over its own (o, n) entries."""
    y, yref = _d(y), _d(yref)
    return np.array([max_abs_rel(y[b], yref[b]) for b in range(y.shape[0])])
