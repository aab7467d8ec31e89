"""MI355X-native explicit LDPM step: HIP library (C-ABI) and its Python binding.

``specimen`` holds the seeded input generator; ``ldpm`` the binding of the
C-ABI library built from ``csrc/``.
"""
