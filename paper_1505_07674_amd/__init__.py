"""MI355X-native forward lensing likelihood (placeholder, binding added below)."""
