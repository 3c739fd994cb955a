"""Helpers for the GPU tests: operator construction from the seeded generator."""
import numpy as np
import torch

import synth
from paper_2608_21763_amd import S2WOperator
from paper_2608_21763_amd.operator import host_generators


def make_operator(cfg, max_batch=1, diff=1, dt=None, chunk_rows=512, **kw):
    dt = cfg.dt if dt is None else dt
    op = S2WOperator(cfg.nsub, cfg.ngrid, cfg.nobs, cfg.nt, max_batch=max_batch, dt=dt, diff=diff, **kw)
    op.load_operators(*host_generators(cfg), chunk_rows=chunk_rows)
    return op


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda:0")


def log_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)
