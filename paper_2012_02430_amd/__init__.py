"""MI355X-native bucket-elimination contractor for QAOA MaxCut tensor networks
with step-dependent slicing (Lykov et al., arXiv 2012.02430).

The contraction runs in ``libqt_hip.so`` (hand-written HIP for gfx950 behind
the C-ABI in ``include/qtensor_hip.h``); this package holds the ctypes
binding (``_lib``), the QAOA network builder (``network``), the Python
wrappers (``api``) and the build script (``build``).
"""
from paper_2012_02430_amd.network import NetworkSpec, amplitude_network, energy_network, edge_lightcone  # noqa: F401
