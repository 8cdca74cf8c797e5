"""MI355X-native exponential-window frequency-domain BEM (arXiv:1212.3032).

The computation lives in the HIP library ``lib/libewbem.so`` (sources in
``csrc/``, C-ABI in ``include/ewbem.h``); ``ewbem`` is its ctypes binding.
"""

from . import ewbem  # noqa: F401
from .ewbem import Context, EwbemError, setup_from_inputs  # noqa: F401
