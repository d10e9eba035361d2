"""MI355X-native CC-MSAV vesicle time step (HIP for gfx950) behind a C ABI.

The compute lives in ``libccmsav.so`` (sources in ``csrc/``, interface in
``include/ccmsav.h``); ``ccmsav`` is its ctypes binding.
"""
