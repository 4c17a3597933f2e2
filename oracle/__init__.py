"""CPU FP64 oracle of the JUMP integrator (test infrastructure only)."""
