"""MI355X-native cellular-automaton TPC track finding (HIP kernels for gfx950 behind a C ABI).

See ``include/tpc_ca.h`` for the ABI and ``tpcca.py`` for the Python binding.
"""
from .tpcca import Context, TpcError, default_params, load, tracks_to_host  # noqa: F401
