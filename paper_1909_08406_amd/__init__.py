"""MI355X-native hot path of the RD3Q41 energy-conserving lattice Boltzmann
method (Kolluru, Atif, Namburi, Ansumali, arXiv:1909.08406).

The compute path is the HIP library ``liblbm.so`` (built from ``csrc/``);
``lbm`` is its thin ctypes binding, with PyTorch supplying device memory and
streams. ``workloads`` generates seeded initial fields.
"""
