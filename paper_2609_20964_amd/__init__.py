"""MI355X-native grid-Poisson SDF reconstruction (Warp-Geo hot path)."""
