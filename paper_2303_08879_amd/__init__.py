"""MI355X-native selective Fock-amplitude library (arXiv:2303.08879 hot path)."""
