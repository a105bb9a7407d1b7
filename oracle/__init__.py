"""FP64 CPU oracle of the Gaussian pointmap rasterizer (test infrastructure only)."""
