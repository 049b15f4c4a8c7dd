"""MI355X-native periodic RPA hot path (chi0 -> Pi -> Tr ln -> quadrature) behind a C-ABI.

The compute path lives in the HIP library ``librpa.so`` built from ``csrc/``; the Python
module ``rpa`` is a thin ctypes binding and ``inputs`` holds the seeded synthetic inputs.
Importing this package loads nothing; ``paper_2505_06021_amd.rpa`` loads the library.
"""
