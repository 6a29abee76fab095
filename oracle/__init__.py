"""CPU oracle for the bitonic sort (test infrastructure only; see oracle.py)."""
