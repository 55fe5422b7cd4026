"""Multidirect-forcing immersed-boundary loop (arXiv 2408.14140) on AMD MI355X.

The work is done by ``libibx.so`` (hand-written HIP for gfx950, C ABI in
``include/ibx.h``); ``ibx`` is its ctypes binding and ``autograd`` wraps the
hand-written adjoint as a ``torch.autograd.Function``.
"""
from .ibx import *  # noqa: F401,F403
from .ibx import (Buckets, DeviceLevel, IbxError, Markers, Particles, Plan, bucket,  # noqa: F401
                  build_markers, count_markers, desired_velocity, device_level, interp,
                  markers_from, particle_reductions, particles, spread)
