"""liblogdet: OSLQ / OSA-IOP log-determinant estimation on one MI355X.

The compute path is the HIP library built from csrc/ (see build.py); this
package only carries its ctypes binding.
"""
from . import liblogdet  # noqa: F401
from .liblogdet import *  # noqa: F401,F403
