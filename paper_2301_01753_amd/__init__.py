"""MI355X-native matrix-free FEEC operators (Q_r^- Lambda^k on hex meshes).

The compute path is the HIP library ``lib/libgym.so`` (C ABI in
``include/gym.h``); :mod:`paper_2301_01753_amd.gym` is its thin ctypes
binding.  PyTorch is used only for device memory and streams.
"""
from . import gym  # noqa: F401
