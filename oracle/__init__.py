"""FP64 CPU oracle for the SORF hot path (test infrastructure only)."""
