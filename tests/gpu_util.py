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


# Half-precision stores.  The bound of the half path is rel-L2 <= 2e-3 per rupture; float16 stores
# meet it everywhere.  Stores with a bfloat16 operator do NOT meet it on dense iid operators
# (measured 2.3-3.9e-3 for bf16/bf16 and 1.7-2.8e-3 for the mixed pairs): their 8-bit mantissa
# rounds each stored value by up to 2^-9 relative, and on incoherent dense data the rounding of
# both operators adds up to about that much in the output.  Those stores are held to a
# regression ceiling of 5e-3 instead, which is not the bound and is reported as not meeting it.
HALF_BOUND = 2e-3
BF16_CEILING = 5e-3


def half_limit(gdt: str, fdt: str) -> float:
    return HALF_BOUND if (gdt, fdt) == ("f16", "f16") else BF16_CEILING


def report_half(label: str, rel: np.ndarray, mabs: np.ndarray) -> None:
    """Print per-rupture rel-L2 and element-wise errors and whether the 2e-3 bound is met."""
    met = "meets" if rel.max() <= HALF_BOUND else "does NOT meet"
    print(f"{label}: rel-L2 max {rel.max():.2e} p50 {np.median(rel):.2e}, element-wise max {mabs.max():.2e}; "
          f"{met} the 2e-3 bound", flush=True)
