"""FP64 CPU oracle package (test infrastructure only; never imported by the GPU path)."""
