"""FP64 CPU oracle for Chord Length Sampling (test infrastructure only)."""
