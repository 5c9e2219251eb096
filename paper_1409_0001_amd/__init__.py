"""MI355X-native diffusion-based coarse graining (placeholder; binding below)."""
