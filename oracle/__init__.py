"""FP64 CPU oracle of the GLM-MHD block update (test infrastructure only)."""
