"""MI355X-native D2V19 + WENO5 finite-difference lattice-Boltzmann step.

The compute path lives in the HIP library ``liblbm_hip.so`` behind the C-ABI
declared in ``include/lbm.h``; ``paper_1010_4124_amd.lbm`` is its thin ctypes
binding. ``paper_1010_4124_amd.inputs`` holds the seeded workload recipes.
Submodules are imported on demand so that the input recipes can be used
without a GPU.
"""
__all__ = ["lbm", "inputs"]
