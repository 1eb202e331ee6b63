"""FP64 CPU oracle for the beamforming product (test infrastructure only)."""
