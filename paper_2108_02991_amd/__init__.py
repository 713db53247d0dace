"""MI355X-native hot path of full-3D SPARKLING (energy, gradient, projection, step)."""
