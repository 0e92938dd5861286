"""CPU FP64 oracle of RSRR and its independent pins (test infrastructure only)."""
