"""MI355X (gfx950) GSIS kinetic hot path: HIP kernels behind a C-ABI (libgsis.so)."""
