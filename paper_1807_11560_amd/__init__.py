"""MI355X-native band-limited Jacobi PDE-EPDiff LDDMM (arXiv 1807.11560).

The compute path is the HIP library ``liblddmm.so`` built from ``csrc/``; the
Python binding in ``lddmm.py`` only marshals arguments to its C-ABI.
``synth`` generates seeded synthetic workloads.
"""
