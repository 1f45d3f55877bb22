"""MI355X-native state-vector quantum circuit simulator (HIP, gfx950).

The public surface is the C ABI in include/qsim.h; ``qsim`` is its ctypes
binding.
"""
from . import qsim  # noqa: F401
from .qsim import State, QsimError, schedule, gate_array, run_opts  # noqa: F401
