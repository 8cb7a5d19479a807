"""CPU oracle for the state-vector method (test infrastructure only)."""
