"""MI355X-native layered-medium FMM + GMRES for 2D Helmholtz scattering.

The compute path is the C-ABI library ``liblmfmm.so`` (hand-written HIP
kernels for gfx950 plus its native host runtime); ``lmfmm`` is the thin
ctypes binding and ``workloads`` generates seeded synthetic inputs.
"""
