"""MI355X-native two-component Shan-Chen D3Q19 lattice Boltzmann with moving
ellipsoidal particles (arXiv:1109.3277).

The compute path is the HIP library ``liblbe.so`` built from ``csrc/``; the
Python binding in ``binding.py`` only marshals arguments through its C ABI.
Seeded synthetic inputs live in ``workloads.py``.
"""
