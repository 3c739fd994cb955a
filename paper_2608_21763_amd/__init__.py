"""MI355X-native source-to-waveform map (one GPU's share of the seafloor grid).

The GPU work lives in ``libs2w.so`` (hand-written gfx950 HIP kernels behind the
C-ABI declared in ``include/s2w.h``); this package only marshals arguments.
``S2WOperator`` owns the device memory (allocated with PyTorch) and
``SourceToWaveform`` exposes the map to ``torch.autograd``.
"""
from .abi import S2WError, Plan, Bltt, load_library, DTYPES, DIFF_NONE, DIFF_BACKWARD  # noqa: F401
from .operator import S2WOperator, SourceToWaveform, source_to_waveform, BLTTOperator  # noqa: F401
from .sizes import spectral_store_bytes, algorithmic_bytes  # noqa: F401
from .autotune import autotune  # noqa: F401
