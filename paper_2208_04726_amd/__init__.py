"""MI355X-native bundle adjustment for Deep Patch Visual Odometry (arXiv 2208.04726)."""
