"""FP64 CPU oracle for the growing-tissue D2Q9 LBM (test infrastructure only)."""
