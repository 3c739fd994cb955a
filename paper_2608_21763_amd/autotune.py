"""Tile-shape autotuner for an ``S2WOperator``.

Times every candidate kernel shape of the operator's path for a batch of B ruptures with
HIP events on the current stream and keeps the fastest through ``s2w_set_tuning``.

What a choice changes in the numbers: the elastic GEMM tiles of the half-precision path,
and the float32 tiles, accumulate every output over the same K steps in the same order, so
they give bit-identical results (tested).  The split counts over grid rows are left on their
defaults, but those defaults follow the tile: the acoustic kernel choice (``fgemm_lds``)
sets how many column tiles the acoustic GEMM has and the adjoint's tiles (``hadj_tile_*``)
how many tiles the elastic transpose has, and from those the number of grid-row ranges
summed in fixed order.  A tuned configuration can therefore sum the grid rows in a
different grouping than the default one and differ from it by rounding (2e-6 relative
at B = 256 on the Cascadia-sized share); the tests cover both groupings against the oracle.

Results can be cached in a JSON file keyed by the problem shape, the dtypes, the layout,
B and the device name, so that a later process applies the stored choice without timing.
"""
from __future__ import annotations

import itertools
import json
import os

import torch

from .hiprt import HipEvent


def candidates(op, adjoint: bool = False) -> list[dict]:
    """Tuning dictionaries worth timing for this operator's path (forward, or adjoint)."""
    if op.plan_layout() == "direct":
        return [{}]  # the direct layout has no tile controls
    if adjoint:
        if op.g_dtype != "f32":
            return [{"hadj_tile_f": a, "hadj_tile_g": b} for a, b in itertools.product((3, 4, 6, 7, 8), repeat=2)]
        if op.plan_layout() == "batched":
            return [{"adj32_cfg": a} for a in (1, 2, 3, 4)]
        return [{"fused_rows": r, "fused_wg_per_cu": w} for r in (4, 8) for w in (1, 2)]
    if op.g_dtype != "f32":
        return [{"gemm_cfg": g, "fgemm_lds": f} for g in (4, 10, 12, 16, 17, 18, 24) for f in (3, 4, 2)]
    if op.plan_layout() == "batched":
        return [{"gemm32_cfg": a, "gemm32_cfg_k": b} for a, b in itertools.product((1, 2, 3, 4), repeat=2)]
    return [{"fused_rows": r, "fused_wg_per_cu": w} for r in (4, 8) for w in (1, 2)]


def _key(op, B: int) -> str:
    name = torch.cuda.get_device_name(op.device)
    return (f"{name}|{op.nsub}x{op.ngrid}x{op.nobs}x{op.nt}|{op.g_dtype}/{op.f_dtype}|{op.plan_layout()}|B={B}"
            f"|diff={op.diff}")


def _time(op, fn, reps: int) -> float:
    stream = torch.cuda.current_stream(op.device).cuda_stream
    fn()  # warm-up (first launch of each kernel shape)
    best = float("inf")
    for _ in range(reps):
        t0, t1 = HipEvent(), HipEvent()
        t0.record(stream)
        fn()
        t1.record(stream)
        t1.synchronize()
        best = min(best, t0.elapsed_ms(t1))
    return best


def autotune(op, B: int, reps: int = 3, adjoint: bool | None = None, cache_path: str | None = None,
             s: torch.Tensor | None = None) -> dict:
    """Pick the fastest tile shapes of ``op`` for batches of B and apply them.

    The objective is the time of one forward call, plus one adjoint call when ``adjoint``
    is true (the default); the adjoint's own tiles (half-precision stores: both products;
    float32 batched layout: the transposed elastic product) are tuned on the adjoint's time.  Returns
    ``{"best": tuning, "ms": time, "results": [(tuning, ms), ...], "cached": bool}``.
    """
    if not 1 <= B <= op.max_batch:
        raise ValueError(f"B={B} outside [1, {op.max_batch}]")
    key = _key(op, B)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            op.set_tuning(**cache[key]["best"])
            return dict(cache[key], cached=True)
    if adjoint is None:
        adjoint = True
    dev = op.device
    if s is None:
        s = torch.randn((B, op.nsub, op.nt), device=dev, dtype=torch.float32)
    y = torch.empty((B, op.nobs, op.nt), device=dev, dtype=torch.float32)
    r = torch.randn((B, op.nobs, op.nt), device=dev, dtype=torch.float32) if adjoint else None
    gs = torch.empty((B, op.nsub, op.nt), device=dev, dtype=torch.float32) if adjoint else None
    base = op.get_tuning()

    def fwd():
        op.forward(s, out=y)

    def adj():
        op.adjoint(r, out=gs)

    def both():
        fwd()
        adj()

    if adjoint and op.g_dtype != "f32":
        # the half-precision adjoint has tile controls of its own: tune the two calls apart
        phases = [(candidates(op), fwd), (candidates(op, adjoint=True), adj)]
    elif adjoint and op.plan_layout() == "batched":
        # float32: the grid-row tile serves the forward elastic and the adjoint acoustic product,
        # so it is tuned on both calls; the adjoint's elastic product then on the adjoint alone
        phases = [(candidates(op), both), (candidates(op, adjoint=True), adj)]
    else:
        # the single layout's controls serve the forward and the adjoint alike
        phases = [(candidates(op), both if adjoint else fwd)]
    results, best, ms = [], {}, 0.0
    for cands, call in phases:
        timed = []
        for cand in cands:
            op.set_tuning(**cand)
            timed.append((cand, _time(op, call, reps)))
        pbest, pms = min(timed, key=lambda t: t[1])
        op.set_tuning(**{k: base[k] for k in pbest})
        op.set_tuning(**pbest)
        results += timed
        best.update(pbest)
        ms += pms
    out = {"best": best, "ms": ms, "results": results, "cached": False}
    if cache_path:
        cache[key] = {"best": best, "ms": ms, "results": results}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    return out
