"""MI355X-native IFEM coupling step (arXiv 1807.08219)."""
