"""FP64 CPU oracle for radiomic spatial mapping (test infrastructure only)."""
