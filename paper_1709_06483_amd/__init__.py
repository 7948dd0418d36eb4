"""MI355X-native Magnus-Leja propagation of the discrete Schroedinger equation.

The hot path (Leja-interpolated actions of matrix exponentials inside fourth
order Magnus steps, Auer, Einkemmer, Kandolf and Ostermann, arXiv 1709.06483)
lives in hand-written HIP kernels behind the C ABI declared in
``include/magnus.h``.  ``binding`` is the thin ctypes layer over that library;
``inputs`` builds the seeded synthetic spin Hamiltonians and states.

Importing this package loads nothing native: ``binding`` opens the shared
library on first use and raises if it has not been built.
"""

__all__ = ["inputs", "binding"]
