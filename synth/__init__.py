"""Seeded synthetic inputs for the source-to-waveform map.

Generates subfault / seafloor-grid / observer positions, time-domain elastic
response blocks G[g][j][k] = [F_{G,k}]_{g,j} (paper Sec. II-B1, eq. 1),
time-domain acoustic-gravity response blocks F[g][o][k] = [F_{q,k}]_{o,g}
(Sec. II-B2, eq. 2), slip-rate histories and observation noise.  Every value
is a pure function of a seed and its indices (a counter-based generator in
``s2w_synth.c``), so grid-row chunks and column subsets regenerate
bit-identically.  This module holds none of the method's arithmetic; the FP64
oracle and the GPU library's callers both draw their inputs from it.

Workload presets follow the paper's Cascadia shapes (Sec. III-C, Table II):
963 subfaults, a 1/64 share (37,760 rows) of the 2,416,530-point seafloor
grid, 64 observers, 256 one-second steps.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libs2w_synth.so")
_SRC = os.path.join(_HERE, "s2w_synth.c")

TAG_VEC_STREAMS = {"x": 1, "y": 2, "r": 3}


def build(verbose: bool = False) -> str:
    """Compile the generator into ``libs2w_synth.so`` (gcc, OpenMP)."""
    import subprocess
    cmd = ["gcc", "-O3", "-mavx2", "-mfma", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-std=c99", "-Wall", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("nsub", ctypes.c_int64), ("ngrid", ctypes.c_int64), ("nobs", ctypes.c_int64), ("nt", ctypes.c_int64),
        ("dt", ctypes.c_double), ("seed", ctypes.c_uint64), ("slip_seed", ctypes.c_uint64),
        ("op_kind", ctypes.c_int32), ("slip_mode", ctypes.c_int32),
        ("box_x", ctypes.c_double), ("box_y", ctypes.c_double),
        ("v_g", ctypes.c_double), ("v_f", ctypes.c_double), ("decay_km", ctypes.c_double),
        ("tau_lo", ctypes.c_double), ("tau_hi", ctypes.c_double),
        ("f_lo", ctypes.c_double), ("f_hi", ctypes.c_double),
        ("v_rup", ctypes.c_double), ("w_lo", ctypes.c_double), ("w_hi", ctypes.c_double),
        ("len_lo", ctypes.c_double), ("len_hi", ctypes.c_double), ("k_lo", ctypes.c_int64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        lib.s2w_synth_G.argtypes = [P(_Cfg), ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_void_p]
        lib.s2w_synth_F.argtypes = [P(_Cfg), ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
        lib.s2w_synth_slip.argtypes = [P(_Cfg), ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        lib.s2w_synth_positions.argtypes = [P(_Cfg), ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_void_p]
        lib.s2w_synth_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_void_p]
        lib.s2w_synth_noise.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p]
        lib.s2w_synth_uniform.restype = ctypes.c_double
        lib.s2w_synth_uniform.argtypes = [ctypes.c_uint64] * 5
        lib.s2w_synth_normal.restype = ctypes.c_double
        lib.s2w_synth_normal.argtypes = [ctypes.c_uint64] * 5
        _lib = lib
    return _lib


@dataclasses.dataclass(frozen=True)
class SynthConfig:
    """Shape and distribution of one synthetic workload.

    op_kind: "physical" (damped sinusoid with spatial decay and travel-time
    onset) or "dense" (iid N(0,1) at every lag).  slip_mode: "all" (every
    subfault active, width w_lo), "length" (active within half a rupture
    length drawn from U(len_lo, len_hi) km of the hypocentre), "knearest"
    (K ~ U{k_lo..nsub} subfaults nearest the hypocentre, width U(w_lo, w_hi))
    or "dense" (iid N(0,1)).
    """
    nsub: int
    ngrid: int
    nobs: int
    nt: int
    dt: float = 1.0
    seed: int = 26080
    slip_seed: int = 26080
    op_kind: str = "physical"
    slip_mode: str = "all"
    box_x: float = 100.0
    box_y: float = 200.0
    v_g: float = 3.0
    v_f: float = 0.2
    decay_km: float = 30.0
    tau_lo: float = 3.0
    tau_hi: float = 10.0
    f_lo: float = 0.05
    f_hi: float = 0.3
    v_rup: float = 2.5
    w_lo: float = 4.0
    w_hi: float = 4.0
    len_lo: float = 50.0
    len_hi: float = 400.0
    k_lo: int = 20

    def replace(self, **kw) -> "SynthConfig":
        return dataclasses.replace(self, **kw)

    def _c(self) -> _Cfg:
        return _Cfg(self.nsub, self.ngrid, self.nobs, self.nt, self.dt, self.seed, self.slip_seed,
                    {"physical": 0, "dense": 1}[self.op_kind],
                    {"all": 0, "length": 1, "knearest": 2, "dense": 3}[self.slip_mode],
                    self.box_x, self.box_y, self.v_g, self.v_f, self.decay_km, self.tau_lo, self.tau_hi,
                    self.f_lo, self.f_hi, self.v_rup, self.w_lo, self.w_hi, self.len_lo, self.len_hi, self.k_lo)


MASTER_SEED = 26080


def workload(name: str) -> SynthConfig:
    """Named workloads.

    small          16 x 512 x 4 x 32, 100 x 200 km box, all subfaults active, W = 4 s
    small_dense    same sizes, iid N(0,1) operators and slip
    cascadia       963 x 37,760 x 64 x 256 (a 1/64 share of 2,416,530 grid points),
                   1000 x 150 km strip, rupture length U(50, 400) km, W = 4 s
    cascadia_batch same operators; K ~ U{20..963} active subfaults, W ~ U(2, 10) s
    cascadia_x2    963 x 75,520 x 64 x 256 (a 1/32 share), batch slip as above
    cascadia_adj   cascadia operators; batch slip; used for the misfit gradient
    strong_p8      60 x 302,067 x 4 x 256: one of eight GPUs' shares of the strong-scaling
                   problem (60 subfaults, 4 observers, all 2,416,530 grid points), Table I
    weak           480 x 37,758 x 32 x 256: one GPU's share of the weak-scaling problem, Table I
    """
    small = SynthConfig(nsub=16, ngrid=512, nobs=4, nt=32, seed=MASTER_SEED, slip_seed=MASTER_SEED)
    strip = dict(box_x=1000.0, box_y=150.0, seed=MASTER_SEED + 1)
    if name == "small":
        return small
    if name == "small_dense":
        return small.replace(op_kind="dense", slip_mode="dense", seed=MASTER_SEED + 10, slip_seed=MASTER_SEED + 10)
    if name == "cascadia":
        return SynthConfig(nsub=963, ngrid=37760, nobs=64, nt=256, slip_mode="length", slip_seed=MASTER_SEED + 1,
                           **strip)
    if name == "cascadia_batch":
        return SynthConfig(nsub=963, ngrid=37760, nobs=64, nt=256, slip_mode="knearest", w_lo=2.0, w_hi=10.0,
                           slip_seed=MASTER_SEED + 2, **strip)
    if name == "cascadia_x2":
        return SynthConfig(nsub=963, ngrid=75520, nobs=64, nt=256, slip_mode="knearest", w_lo=2.0, w_hi=10.0,
                           slip_seed=MASTER_SEED + 3, **strip)
    if name == "cascadia_adj":
        return SynthConfig(nsub=963, ngrid=37760, nobs=64, nt=256, slip_mode="knearest", w_lo=2.0, w_hi=10.0,
                           slip_seed=MASTER_SEED + 4, **strip)
    if name == "strong_p8":
        return SynthConfig(nsub=60, ngrid=302067, nobs=4, nt=256, slip_mode="length", slip_seed=MASTER_SEED + 5,
                           **strip)
    if name == "weak":
        return SynthConfig(nsub=480, ngrid=37758, nobs=32, nt=256, slip_mode="length", slip_seed=MASTER_SEED + 6,
                           **strip)
    raise KeyError(name)


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def gen_G(cfg: SynthConfig, row0: int = 0, nrows: int | None = None, cols=None, out: np.ndarray | None = None):
    """Elastic blocks, float32 [nrows][ncols][nt]; cols=None means all subfaults."""
    lib = _load()
    if nrows is None:
        nrows = cfg.ngrid - row0
    c = cfg._c()
    if cols is None:
        ncols, cptr = cfg.nsub, None
    else:
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        ncols, cptr = len(cols), _ptr(cols)
    if out is None:
        out = np.empty((nrows, ncols, cfg.nt), dtype=np.float32)
    assert out.shape == (nrows, ncols, cfg.nt) and out.dtype == np.float32
    lib.s2w_synth_G(ctypes.byref(c), row0, nrows, cptr, ncols, _ptr(out))
    return out


def gen_F(cfg: SynthConfig, row0: int = 0, nrows: int | None = None, out: np.ndarray | None = None):
    """Acoustic-gravity blocks, float32 [nrows][nobs][nt]."""
    lib = _load()
    if nrows is None:
        nrows = cfg.ngrid - row0
    if out is None:
        out = np.empty((nrows, cfg.nobs, cfg.nt), dtype=np.float32)
    assert out.shape == (nrows, cfg.nobs, cfg.nt) and out.dtype == np.float32
    c = cfg._c()
    lib.s2w_synth_F(ctypes.byref(c), row0, nrows, _ptr(out))
    return out


def gen_slip(cfg: SynthConfig, rup: int, with_info: bool = False):
    """Slip-rate history of rupture `rup`, float32 [nsub][nt]."""
    lib = _load()
    out = np.empty((cfg.nsub, cfg.nt), dtype=np.float32)
    info = np.zeros(4, dtype=np.float64)
    c = cfg._c()
    lib.s2w_synth_slip(ctypes.byref(c), rup, _ptr(out), _ptr(info))
    if with_info:
        return out, {"hypocentre": int(info[0]), "active": int(info[1]), "width_s": float(info[2]),
                     "extent": float(info[3])}
    return out


def gen_slip_batch(cfg: SynthConfig, first: int, count: int) -> np.ndarray:
    """Ruptures first..first+count-1, float32 [count][nsub][nt]."""
    return np.stack([gen_slip(cfg, first + b) for b in range(count)]) if count else \
        np.zeros((0, cfg.nsub, cfg.nt), np.float32)


def positions(cfg: SynthConfig, kind: str, i0: int = 0, n: int | None = None) -> np.ndarray:
    """(x, y) in km, float64 [n][2]; kind in {"sub", "grid", "obs"}."""
    lib = _load()
    k = {"sub": 0, "grid": 1, "obs": 2}[kind]
    total = {"sub": cfg.nsub, "grid": cfg.ngrid, "obs": cfg.nobs}[kind]
    if n is None:
        n = total - i0
    out = np.empty((n, 2), dtype=np.float64)
    c = cfg._c()
    lib.s2w_synth_positions(ctypes.byref(c), k, i0, n, _ptr(out))
    return out


def normals(seed: int, stream: str, idx: int, shape) -> np.ndarray:
    """iid N(0,1) float64 array of `shape` from a named stream ("x", "y", "r")."""
    lib = _load()
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.float64)
    lib.s2w_synth_normals(seed, TAG_VEC_STREAMS[stream], idx, n, _ptr(out))
    return out.reshape(shape)


def noise(seed: int, shape) -> np.ndarray:
    """iid N(0,1) observation noise, float64."""
    lib = _load()
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.float64)
    lib.s2w_synth_noise(seed, n, _ptr(out))
    return out.reshape(shape)


def active_columns(slips: np.ndarray) -> np.ndarray:
    """Subfault indices whose slip-rate is nonzero in any of the given ruptures."""
    s = np.asarray(slips).reshape(-1, slips.shape[-2], slips.shape[-1])
    return np.nonzero(np.any(s != 0, axis=(0, 2)))[0].astype(np.int64)
