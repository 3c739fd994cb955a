"""Host-side logic and the C-ABI library, without a GPU."""
import ctypes
import json
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    from paper_2608_21763_amd import abi
    header = open(os.path.join(ROOT, "include", "s2w.h")).read()
    declared = set(re.findall(r"^\s*(?:s2w_status|const char\*|int32_t)\s+(s2w_\w+)\s*\(", header, re.M))
    assert {"s2w_forward", "s2w_adjoint", "s2w_set_operators", "s2w_plan_create"} <= declared
    lib = ctypes.CDLL(abi.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), f"{name} declared in s2w.h but not exported"
    assert declared == set(abi.EXPORTS)
    assert abi.load_library().s2w_abi_version() == 6


def test_table2_storage_from_byte_calculator():
    # the paper's persistent coefficients: all Nt+1 bins of a length-2Nt FFT, complex128,
    # for (Nf + Nq) columns over one 1/64 share of the grid (the largest share has 37,759 rows)
    from paper_2608_21763_amd import spectral_store_bytes
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "table2_storage.json")))
    share = math.ceil(g["ngrid_total"] / g["gpus"])
    b = spectral_store_bytes(g["nsub"], g["nobs"], share, g["nt"], bytes_per_complex=16)
    assert round(b / 2 ** 30, 2) == g["persistent_gib_per_gpu"]
    assert round(g["resident_gib_per_gpu"] * g["gpus"] / 1024, 2) == g["aggregate_tib"]
    assert g["ngrid_total"] * g["nt"] == g["seafloor_field_dimension"]


def test_algorithmic_bytes_of_the_share():
    from paper_2608_21763_amd import algorithmic_bytes, spectral_store_bytes
    # 2*Nt real values per (row, column) pair: the 257 bins with the two real ones packed
    a = algorithmic_bytes(963, 64, 37760, 256, 4)
    assert a == spectral_store_bytes(963, 64, 37760, 256, 8, packed_real_bins=True)
    assert abs(a / 1e9 - 79.43) < 0.01


def test_plan_create_rejects_bad_descriptors_without_gpu():
    from paper_2608_21763_amd import abi
    lib = abi.load_library()
    bad = [dict(nsub=0), dict(nt=513), dict(nobs=257), dict(dt=0.0), dict(diff=3), dict(g_dtype=7), dict(max_batch=-1)]
    for kw in bad:
        d = dict(nsub=16, ngrid=512, nobs=4, nt=32, max_batch=1, diff=1, g_dtype=0, f_dtype=0, dt=1.0)
        d.update(kw)
        desc = abi.Desc(**d)
        h = ctypes.c_void_p()
        st = lib.s2w_plan_create(ctypes.byref(desc), 0, ctypes.byref(h))
        assert st == 1 and not h.value, kw


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stdout


def test_missing_library_fails_loudly(tmp_path):
    # without the built HIP library the package refuses to work instead of falling back
    import subprocess
    import sys
    import textwrap
    code = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {repr(str(ROOT))})
        import paper_2608_21763_amd.abi as abi
        abi.LIB_PATH = {repr(str(tmp_path / 'missing' / 'libs2w.so'))}
        try:
            abi.Plan(4, 8, 2, 16)
        except ImportError as e:
            print("refused:", e)
            sys.exit(0)
        sys.exit(1)
    """)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "refused" in r.stdout
