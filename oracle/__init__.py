"""FP64 CPU oracle of the GSIS kinetic pass (test infrastructure only)."""
