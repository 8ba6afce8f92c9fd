"""MI355X-native real-space DFPT RPA chi0 hot path (arXiv:2504.01816)."""
