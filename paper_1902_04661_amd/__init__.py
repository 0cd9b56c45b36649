"""gqd on MI355X: implicit, exactly unitary geometric integrators for nonadiabatic
quantum dynamics in the adiabatic representation (Choi & Vanicek, J. Chem. Phys.
150, 204112 (2019)), as HIP kernels for gfx950 behind a C ABI (include/gqd.h).

Importing the package loads nothing; `paper_1902_04661_amd.gqd` loads libgqd.so on
first use and raises if it is not built."""

__all__ = ["gqd", "inputs"]
