"""PyTorch-facing wrapper: device memory, streams and autograd around the C-ABI.

PyTorch supplies device memory and the current stream only; every step of the
map runs in the HIP kernels of ``libs2w.so``.
"""
from __future__ import annotations

import numpy as np
import torch

from .abi import DIFF_BACKWARD, Bltt, Plan

_ALIGN = 256


def _aligned(t: torch.Tensor) -> bool:
    return t.data_ptr() % _ALIGN == 0


def _prep(t: torch.Tensor, shape, device) -> torch.Tensor:
    """Contiguous, 256-byte aligned float32 view of `t` on `device` (copies only if needed)."""
    if t.dtype != torch.float32 or t.device != device:
        t = t.to(device=device, dtype=torch.float32)
    if tuple(t.shape) != tuple(shape):
        t = t.reshape(shape)
    if not t.is_contiguous() or not _aligned(t):
        c = torch.empty(shape, dtype=torch.float32, device=device)
        c.copy_(t)
        t = c
    return t


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class S2WOperator:
    """One share of the source-to-waveform map with its operator spectra resident on a GPU.

    Allocates the operator store and workspace with PyTorch, then ``set_operators``
    receives time-domain blocks in grid-row chunks.  ``forward(s)`` returns the
    share's partial waveforms; ``adjoint(r)`` its transpose.
    """

    def __init__(self, nsub: int, ngrid: int, nobs: int, nt: int, max_batch: int = 1, dt: float = 1.0,
                 diff: int = DIFF_BACKWARD, g_dtype: str = "f32", f_dtype: str = "f32", device: int | str = 0,
                 layout: str = "auto", products: str = "auto"):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        idx = self.device.index if self.device.index is not None else torch.cuda.current_device()
        self.nsub, self.ngrid, self.nobs, self.nt, self.max_batch = nsub, ngrid, nobs, nt, max_batch
        self.dt, self.diff, self.g_dtype, self.f_dtype = dt, diff, g_dtype, f_dtype
        self.layout, self.products = layout, products
        self.plan = Plan(nsub, ngrid, nobs, nt, max_batch, dt, diff, g_dtype, f_dtype, idx, layout, products)
        op_bytes, ws_bytes = self.plan.query_sizes()
        self.op_store = torch.empty(max(op_bytes, 1), dtype=torch.uint8, device=self.device)
        self.workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=self.device)
        assert _aligned(self.op_store) and _aligned(self.workspace)
        self.plan.bind(self.op_store.data_ptr(), op_bytes, self.workspace.data_ptr(), ws_bytes)
        self.L = self.plan.transform_length()

    # -- setup -----------------------------------------------------------------------------------
    def set_operators(self, G_chunk: torch.Tensor, F_chunk: torch.Tensor, row0: int):
        """Time-domain blocks of rows [row0, row0 + n): G[n][nsub][nt], F[n][nobs][nt] (device tensors)."""
        n = G_chunk.shape[0]
        G_chunk = _prep(G_chunk, (n, self.nsub, self.nt), self.device)
        F_chunk = _prep(F_chunk, (n, self.nobs, self.nt), self.device)
        self.plan.set_operators(G_chunk.data_ptr(), F_chunk.data_ptr(), row0, n, _stream_handle(self.device))
        return G_chunk, F_chunk  # the caller keeps them alive until the stream passes

    def load_operators(self, gen_G, gen_F, chunk_rows: int = 512, progress=None):
        """Fill every row from host generators ``gen_G(row0, n, out)`` / ``gen_F(row0, n, out)``
        writing float32 numpy arrays; host chunks are staged through pinned memory, double-buffered."""
        cr = min(chunk_rows, self.ngrid)
        pin = [(torch.empty((cr, self.nsub, self.nt), dtype=torch.float32, pin_memory=True),
                torch.empty((cr, self.nobs, self.nt), dtype=torch.float32, pin_memory=True)) for _ in range(2)]
        dev = [(torch.empty((cr, self.nsub, self.nt), dtype=torch.float32, device=self.device),
                torch.empty((cr, self.nobs, self.nt), dtype=torch.float32, device=self.device)) for _ in range(2)]
        events = [None, None]
        stream = torch.cuda.current_stream(self.device)
        for i, r0 in enumerate(range(0, self.ngrid, cr)):
            n = min(cr, self.ngrid - r0)
            k = i % 2
            if events[k] is not None:
                events[k].synchronize()
            hG, hF = pin[k]
            gen_G(r0, n, hG.numpy()[:n])
            gen_F(r0, n, hF.numpy()[:n])
            dG, dF = dev[k]
            dG[:n].copy_(hG[:n], non_blocking=True)
            dF[:n].copy_(hF[:n], non_blocking=True)
            self.plan.set_operators(dG.data_ptr(), dF.data_ptr(), r0, n, stream.cuda_stream)
            ev = torch.cuda.Event()
            ev.record(stream)
            events[k] = ev
            if progress:
                progress(r0 + n, self.ngrid)
        torch.cuda.synchronize(self.device)

    def plan_layout(self) -> str:
        """"single", "batched" or "direct": the storage layout the plan uses."""
        return self.plan.layout()

    def set_tuning(self, **kw):
        self.plan.set_tuning(**kw)

    def get_tuning(self) -> dict:
        return self.plan.get_tuning()

    # -- the map ---------------------------------------------------------------------------------
    def forward(self, s: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """s[B][nsub][nt] (or [nsub][nt]) -> y[B][nobs][nt] on the current stream."""
        squeeze = s.dim() == 2
        B = 1 if squeeze else s.shape[0]
        s = _prep(s, (B, self.nsub, self.nt), self.device)
        y = out if out is not None else torch.empty((B, self.nobs, self.nt), dtype=torch.float32, device=self.device)
        assert y.is_contiguous() and _aligned(y) and y.shape == (B, self.nobs, self.nt)
        self.plan.forward(s.data_ptr(), B, y.data_ptr(), _stream_handle(self.device))
        return y[0] if squeeze else y

    def forward_displacement(self, s: torch.Tensor, times=None):
        """(y, m): the waveforms and the share's seafloor displacement m[B][ngrid][len(times)] at the
        given steps (every step when None), both from one pass of the map."""
        squeeze = s.dim() == 2
        B = 1 if squeeze else s.shape[0]
        s = _prep(s, (B, self.nsub, self.nt), self.device)
        nts = self.nt if times is None else len(times)
        y = torch.empty((B, self.nobs, self.nt), dtype=torch.float32, device=self.device)
        m = torch.empty((B, self.ngrid, nts), dtype=torch.float32, device=self.device)
        self.plan.forward_displacement(s.data_ptr(), B, y.data_ptr(), m.data_ptr(),
                                       None if times is None else list(times), nts, _stream_handle(self.device))
        return (y[0], m[0]) if squeeze else (y, m)

    def adjoint(self, r: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """r[B][nobs][nt] (or [nobs][nt]) -> gs[B][nsub][nt] = A^T r on the current stream."""
        squeeze = r.dim() == 2
        B = 1 if squeeze else r.shape[0]
        r = _prep(r, (B, self.nobs, self.nt), self.device)
        gs = out if out is not None else torch.empty((B, self.nsub, self.nt), dtype=torch.float32, device=self.device)
        assert gs.is_contiguous() and _aligned(gs) and gs.shape == (B, self.nsub, self.nt)
        self.plan.adjoint(r.data_ptr(), B, gs.data_ptr(), _stream_handle(self.device))
        return gs[0] if squeeze else gs

    def __call__(self, s: torch.Tensor) -> torch.Tensor:
        return source_to_waveform(s, self)


class SourceToWaveform(torch.autograd.Function):
    """y = A s with dL/ds = A^T dL/dy through the hand-written adjoint kernels."""

    @staticmethod
    def forward(ctx, s: torch.Tensor, op: S2WOperator):
        ctx.op = op
        return op.forward(s.detach())

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        return ctx.op.adjoint(gy.contiguous()), None


def source_to_waveform(s: torch.Tensor, op: S2WOperator) -> torch.Tensor:
    return SourceToWaveform.apply(s, op)


def host_generators(cfg):
    """(gen_G, gen_F) callables over the seeded generator ``synth`` for ``load_operators``."""
    import synth

    def gG(r0, n, out):
        synth.gen_G(cfg, r0, n, out=out)

    def gF(r0, n, out):
        synth.gen_F(cfg, r0, n, out=out)

    return gG, gF


class BLTTOperator:
    """One block lower-triangular Toeplitz operator y_n = sum_{k<=n} F_k x_{n-k} (Alg. 2 on its own).

    ``F_k`` is ``nrow x ncol``; blocks are set in row chunks ``F[r][c][k]``.  ``apply(x)``
    maps x[B][ncol][nt] to y[B][nrow][nt], ``adjoint(y)`` is its transpose.  With the elastic
    blocks of a share this gives the seafloor displacement (eq. 1); with the acoustic blocks,
    the partial waveforms of a given seafloor motion (eq. 2).
    """

    def __init__(self, nrow: int, ncol: int, nt: int, max_batch: int = 1, device: int | str = 0):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        idx = self.device.index if self.device.index is not None else torch.cuda.current_device()
        self.nrow, self.ncol, self.nt, self.max_batch = nrow, ncol, nt, max_batch
        self.plan = Bltt(nrow, ncol, nt, max_batch, idx)
        op_bytes, ws_bytes = self.plan.query_sizes()
        self.op_store = torch.empty(max(op_bytes, 1), dtype=torch.uint8, device=self.device)
        self.workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=self.device)
        self.plan.bind(self.op_store.data_ptr(), op_bytes, self.workspace.data_ptr(), ws_bytes)

    def set_blocks(self, F_chunk: torch.Tensor, row0: int):
        n = F_chunk.shape[0]
        F_chunk = _prep(F_chunk, (n, self.ncol, self.nt), self.device)
        self.plan.set_blocks(F_chunk.data_ptr(), row0, n, _stream_handle(self.device))
        return F_chunk

    def load_blocks(self, gen, chunk_rows: int = 256):
        """Fill every row from a host generator ``gen(row0, n, out)`` writing float32 [n][ncol][nt]."""
        for r0 in range(0, self.nrow, chunk_rows):
            n = min(chunk_rows, self.nrow - r0)
            h = torch.empty((n, self.ncol, self.nt), dtype=torch.float32, pin_memory=True)
            gen(r0, n, h.numpy())
            d = h.to(self.device, non_blocking=True)
            self.plan.set_blocks(d.data_ptr(), r0, n, _stream_handle(self.device))
            torch.cuda.current_stream(self.device).synchronize()

    def apply(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        squeeze = x.dim() == 2
        B = 1 if squeeze else x.shape[0]
        x = _prep(x, (B, self.ncol, self.nt), self.device)
        y = out if out is not None else torch.empty((B, self.nrow, self.nt), dtype=torch.float32, device=self.device)
        assert y.is_contiguous() and _aligned(y) and y.shape == (B, self.nrow, self.nt)
        self.plan.apply(x.data_ptr(), B, y.data_ptr(), _stream_handle(self.device))
        return y[0] if squeeze else y

    def adjoint(self, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        squeeze = y.dim() == 2
        B = 1 if squeeze else y.shape[0]
        y = _prep(y, (B, self.nrow, self.nt), self.device)
        x = out if out is not None else torch.empty((B, self.ncol, self.nt), dtype=torch.float32, device=self.device)
        assert x.is_contiguous() and _aligned(x) and x.shape == (B, self.ncol, self.nt)
        self.plan.adjoint(y.data_ptr(), B, x.data_ptr(), _stream_handle(self.device))
        return x[0] if squeeze else x
