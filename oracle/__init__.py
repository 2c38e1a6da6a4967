"""CPU oracle of the inpainting hot path (test infrastructure only)."""
