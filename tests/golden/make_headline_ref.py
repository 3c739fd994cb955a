"""Write the FP64 oracle's waveforms for sampled ruptures of the timed batch.

The timed batch is the first 256 ruptures of the Cascadia-sized ensemble workload
(963 x 37,760 x 64 x 256, K ~ U{20..963} nearest subfaults active, pulse width U(2, 10) s).
The sample is every eighth rupture (0, 8, ..., 248) plus the ruptures with the fewest and
the most active subfaults.  Only ``oracle`` and the seeded generator ``synth`` are called;
the output, ``headline_ref.npz``, holds the indices, their active-subfault counts and the
oracle's waveforms rounded to float32 (a relative change of at most 6e-8, far below every
bound it is compared at).

Run from the repository root:  python tests/golden/make_headline_ref.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

BATCH = 256
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "headline_ref.npz")


def sample_indices(s):
    act = np.array([int(np.count_nonzero(np.any(s[b] != 0, axis=1))) for b in range(s.shape[0])])
    pick = sorted(set(range(0, s.shape[0], 8)) | {int(np.argmin(act)), int(np.argmax(act))})
    return np.array(pick, dtype=np.int64), act


def main():
    cfg = synth.workload("cascadia_batch")
    s = synth.gen_slip_batch(cfg, 0, BATCH)
    idx, act = sample_indices(s)
    t = time.time()
    y = oracle.forward_synth(cfg, s[idx], chunk_rows=256)
    print(f"{len(idx)} ruptures in {time.time() - t:.0f} s", flush=True)
    np.savez(OUT, indices=idx, active=act[idx], y=y.astype(np.float32),
             workload=np.array("cascadia_batch"), batch=np.array(BATCH))


if __name__ == "__main__":
    main()
