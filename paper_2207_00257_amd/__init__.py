"""MI355X-native barrier-hoisted normalize (arXiv 2207.00257, Fig. 1)."""
