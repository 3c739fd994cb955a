"""Byte counts of the operator spectra (host arithmetic only).

The paper keeps every temporal FFT bin l = 0..Nt of both response operators
resident (Alg. 2, bins 0..Nt of a length-2Nt transform) for the rank's grid
rows (Sec. II-C).  ``spectral_store_bytes`` counts that store; with complex128
and Nt + 1 = 257 bins it reproduces Table II's 148.51 GiB per GPU.
"""
from __future__ import annotations


def spectral_store_bytes(nsub: int, nobs: int, ngrid: int, nt: int, bytes_per_complex: int = 16,
                         packed_real_bins: bool = False) -> int:
    """Bytes of the frequency-domain blocks of F_G^(r) and F_q^(r) for `ngrid` rows.

    Unpacked: (Nt + 1) complex bins per (row, column) pair.  Packed: the two real
    bins (0 and Nt) share one complex slot, Nt slots per pair.
    """
    bins = nt if packed_real_bins else nt + 1
    return (nsub + nobs) * ngrid * bins * bytes_per_complex


def algorithmic_bytes(nsub: int, nobs: int, ngrid: int, nt: int, bytes_per_real: int = 4) -> int:
    """Operator bytes one application of the map must read: 2*Nt real numbers
    (Nt - 1 complex bins plus two real bins) per (row, column) pair of each operator."""
    return (nsub + nobs) * ngrid * (2 * nt) * bytes_per_real
