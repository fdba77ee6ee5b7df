"""MI355X-native polynomial-kernel Gaussian splatting (placeholder)."""
