"""bchnms: enhanced normalized min-sum decoding of short BCH codes on AMD
MI355X (gfx950), after Li & Yu, arXiv 2412.20828.

The compute path is the HIP library ``libbchnms.so`` built from ``csrc/``; the
Python layer in ``binding`` only marshals arguments to its C-ABI.
"""
